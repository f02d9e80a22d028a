// Build stage of the hierarchical solver (FP64, once per plan): assembly of
// the element systems, the element Dirichlet-to-Neumann maps and the
// gathers that set up each merge.  The dense factorisations and products
// between these steps are rocSOLVER / rocBLAS calls made by the host code.
#include "hx_kernels.h"

namespace hx {

// Side s (0 left, 1 right, 2 bottom, 3 top) of the slot-th present side.
__device__ __forceinline__ int nth_side(int mask, int slot) {
  int seen = -1;
  for (int k = 0; k < 4; ++k)
    if ((mask >> k) & 1)
      if (++seen == slot) return k;
  return -1;
}

// Element system for shift sigma (block = leaf, chunk pole):
//   A_ii (q^2 x q^2) into the workspace, [I | A_ie] into the operator slot,
// with A = sx^2 Dx C^2 Dx + sy^2 Dy C^2 Dy - sigma on the interior rows.
__global__ __launch_bounds__(kBlock) void k_leaf_assemble(LeafAssembleArgs a) {
  __shared__ double Ds[kMaxP * kMaxP];
  __shared__ double cs[kMaxP * kMaxP];
  const int leaf = blockIdx.x % a.n_leaf;
  const int j = blockIdx.x / a.n_leaf;
  const int p = a.p, q = a.q, q2 = q * q;
  const LeafDesc L = a.leaves[leaf];
  for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
    Ds[t] = a.D[t];
    cs[t] = a.c2[(long long)L.elem * p * p + t];
  }
  __syncthreads();
  const double sx2 = a.sx * a.sx, sy2 = a.sy * a.sy;
  // x part on row jj: sum_m D[i][m] c(m, jj) D[m][k];  y part on column i.
  auto mx = [&](int jj, int i, int k) {
    double s = 0.0;
    for (int m = 0; m < p; ++m) s += Ds[i * p + m] * cs[m + p * jj] * Ds[m * p + k];
    return sx2 * s;
  };
  auto my = [&](int i, int jj, int l) {
    double s = 0.0;
    for (int m = 0; m < p; ++m) s += Ds[jj * p + m] * cs[i + p * m] * Ds[m * p + l];
    return sy2 * s;
  };
  const double2 sg = a.sigma[j];
  double2* A = a.A + ((long long)j * a.n_leaf + leaf) * q2 * q2;
  double2* R = a.ops + j * a.pole_stride + L.op_off;
  for (int f = threadIdx.x; f < q2 * q2; f += blockDim.x) {
    const int c = f / q2, r = f - c * q2;
    const int i = r % q + 1, jj = r / q + 1;
    const int k = c % q + 1, l = c / q + 1;
    double v = 0.0;
    if (l == jj) v += mx(jj, i, k);
    if (k == i) v += my(i, jj, l);
    A[f] = (r == c) ? make_double2(v - sg.x, -sg.y) : make_double2(v, 0.0);
    R[f] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  for (int f = threadIdx.x; f < q2 * L.e; f += blockDim.x) {
    const int c = f / q2, r = f - c * q2;
    const int s = nth_side(L.side_mask, c / q), t = c % q;
    const int i = r % q + 1, jj = r / q + 1;
    double v = 0.0;
    if (s == 0 && jj == t + 1) v = mx(jj, i, 0);
    if (s == 1 && jj == t + 1) v = mx(jj, i, p - 1);
    if (s == 2 && i == t + 1) v = my(i, jj, 0);
    if (s == 3 && i == t + 1) v = my(i, jj, p - 1);
    R[(long long)q2 * q2 + f] = make_double2(v, 0.0);
  }
}

// Element DtN map T = N_e - N_i S (block = leaf, chunk pole), e x e.
__global__ __launch_bounds__(kBlock) void k_leaf_dtn(LeafDtnArgs a) {
  const int leaf = blockIdx.x % a.n_leaf;
  const int j = blockIdx.x / a.n_leaf;
  const int p = a.p, q = a.q, q2 = q * q;
  const LeafDesc L = a.leaves[leaf];
  const int e = L.e;
  const double2* S = a.ops + j * a.pole_stride + L.op_off + (long long)q2 * q2;
  double2* T = a.T + j * a.T_stride + a.T_off[leaf];
  for (int f = threadIdx.x; f < e * e; f += blockDim.x) {
    const int c = f / e, r = f - c * e;
    const int sr = nth_side(L.side_mask, r / q), tr = r % q;
    const int sc = nth_side(L.side_mask, c / q), tc = c % q;
    const bool xn = sr < 2;
    const bool lo = (sr == 0 || sr == 2);
    const double sgn = xn ? (lo ? -a.sx : a.sx) : (lo ? -a.sy : a.sy);
    const double* Dr = a.D + (lo ? 0 : (p - 1)) * p;
    double ne = 0.0;
    if (tc == tr) {
      if (sc == (xn ? 0 : 2)) ne += sgn * Dr[0];
      if (sc == (xn ? 1 : 3)) ne += sgn * Dr[p - 1];
    }
    double2 acc = make_double2(0.0, 0.0);
    const double2* Sc = S + (long long)c * q2;
    for (int k = 1; k <= q; ++k) {
      const int node = xn ? ((k - 1) + q * tr) : (tr + q * (k - 1));
      acc.x += Dr[k] * Sc[node].x;
      acc.y += Dr[k] * Sc[node].y;
    }
    T[f] = make_double2(ne - sgn * acc.x, -sgn * acc.y);
  }
}

// Merge set-up (block = box, chunk pole): M = T33a + T33b, the right-hand
// side [B | I] in the Z slot, V = [T13a; T23b] and diag(T11a, T22b).
__global__ __launch_bounds__(kBlock) void k_merge_gather(MergeGatherArgs a) {
  const int nb = gridDim.x / a.chunk;
  const int box = blockIdx.x % nb;
  const int j = blockIdx.x / nb;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  const int ea = n1 + n3, eb = n2 + n3;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const double2* Ta = a.Tc + j * a.Tc_stride + a.Tc_off[B.a_box];
  const double2* Tb = a.Tc + j * a.Tc_stride + a.Tc_off[B.b_box];
  double2* M = a.M + j * a.M_stride + a.M_off[box];
  for (int f = threadIdx.x; f < n3 * n3; f += blockDim.x) {
    const int c = f / n3, r = f - c * n3;
    const double2 x = Ta[i3a[r] + (long long)i3a[c] * ea];
    const double2 y = Tb[i3b[r] + (long long)i3b[c] * eb];
    M[f] = make_double2(x.x + y.x, x.y + y.y);
  }
  double2* Z = a.ops + j * a.pole_stride + B.op_off;
  for (int f = threadIdx.x; f < n3 * (ext + n3); f += blockDim.x) {
    const int c = f / n3, r = f - c * n3;
    double2 v;
    if (c < n1) v = Ta[i3a[r] + (long long)i1[c] * ea];
    else if (c < ext) v = Tb[i3b[r] + (long long)i2[c - n1] * eb];
    else v = make_double2(r == c - ext ? 1.0 : 0.0, 0.0);
    Z[f] = v;
  }
  if (ext == 0) return;
  double2* V = a.V + j * a.V_stride + a.V_off[box];
  for (int f = threadIdx.x; f < ext * n3; f += blockDim.x) {
    const int c = f / ext, r = f - c * ext;
    V[f] = (r < n1) ? Ta[i1[r] + (long long)i3a[c] * ea] : Tb[i2[r - n1] + (long long)i3b[c] * eb];
  }
  double2* Tp = a.Tp + j * a.Tp_stride + a.Tp_off[box];
  for (int f = threadIdx.x; f < ext * ext; f += blockDim.x) {
    const int c = f / ext, r = f - c * ext;
    double2 v = make_double2(0.0, 0.0);
    if (r < n1 && c < n1) v = Ta[i1[r] + (long long)i1[c] * ea];
    else if (r >= n1 && c >= n1) v = Tb[i2[r - n1] + (long long)i2[c - n1] * eb];
    Tp[f] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_nonfinite(const double* __restrict__ x, long long n,
                                                      int* flag) {
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;
}

// FP64 -> FP32 copy of a chunk of operators (precision form).
__global__ __launch_bounds__(kBlock) void k_pack_f32(const double2* __restrict__ src,
                                                     float2* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 v = src[i];
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

// n x n identity (the right-hand side of a batched inversion).
__global__ __launch_bounds__(kBlock) void k_eye(double2* __restrict__ X, int n) {
  const long long nn = (long long)n * n;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nn;
       f += (long long)gridDim.x * blockDim.x)
    X[f] = make_double2((f % (n + 1)) == 0 ? 1.0 : 0.0, 0.0);
}

hipError_t launch_eye(double2* X, int n, hipStream_t s) {
  long long blocks = ((long long)n * n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_eye, dim3((unsigned)blocks), dim3(kBlock), 0, s, X, n);
  return hipGetLastError();
}

hipError_t launch_pack_f32(const double2* src, float2* dst, long long n, hipStream_t s) {
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_pack_f32, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_leaf_assemble(const LeafAssembleArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_assemble, dim3(a.n_leaf * a.chunk), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_leaf_dtn(const LeafDtnArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_dtn, dim3(a.n_leaf * a.chunk), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_merge_gather(const MergeGatherArgs& a, int n_box, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_gather, dim3(n_box * a.chunk), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nonfinite_check(const double* x, long long n, int* flag, hipStream_t s) {
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, n, flag);
  return hipGetLastError();
}

}  // namespace hx
