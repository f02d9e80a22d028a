// Solve-stage sweeps of the hierarchical solver, FP64 complex, one
// right-hand side per column (column c = pole * nrhs + rhs), and the pole
// sum of the rational time step.
//
// Every operator is a dense complex matrix stored column-major and read
// exactly once per column per step: each kernel is a batch of complex
// matrix-vector products, bound by HBM bandwidth.  A thread owns one
// output row and walks the columns, so a wavefront reads 64 consecutive
// rows of one column (1 KiB contiguous) per load; the input vector sits
// in LDS and is broadcast.
#include "hx_kernels.h"

namespace hx {

__device__ __forceinline__ void cfma(double2& acc, const double2 a, const double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

typedef double v2d __attribute__((ext_vector_type(2)));

// Streaming load of one complex operator entry (read once per step, so it
// is marked non-temporal to keep it from displacing reused vectors).
__device__ __forceinline__ double2 ldnt(const double2* p) {
  const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
  return make_double2(v.x, v.y);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}

// Column-major matrix-vector product over the row block [r0, r0 + nr):
//   out[t] = sum_{c < m} A[(r0 + t) + c*lda] x[c],  valid in thread t < nr.
// The BS threads split into G = BS / nr column groups (G = 1 for tall
// blocks), so short operators still keep every lane loading: group g reads
// columns g, g+G, ...; at each step the block reads G*nr consecutive entries
// when nr is the whole column.  Partials are summed through LDS in a fixed
// order.  Must be called by every thread of the block.
template <int BS>
__device__ __forceinline__ double2 gemv_cm(const double2* __restrict__ A, long long lda, int r0,
                                           int nr, int m, const double2* __restrict__ x,
                                           double2* __restrict__ red) {
  const int t = threadIdx.x;
  const int G = nr >= BS ? 1 : BS / nr;
  const int g = t / nr, r = t - g * nr;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  if (g < G) {
    const double2* Ar = A + r0 + r;
    int c = g;
    for (; c + 3 * G < m; c += 4 * G) {
      const double2 m0 = ldnt(Ar + (long long)c * lda);
      const double2 m1 = ldnt(Ar + (long long)(c + G) * lda);
      const double2 m2 = ldnt(Ar + (long long)(c + 2 * G) * lda);
      const double2 m3 = ldnt(Ar + (long long)(c + 3 * G) * lda);
      cfma(a0, m0, x[c]);
      cfma(a1, m1, x[c + G]);
      cfma(a0, m2, x[c + 2 * G]);
      cfma(a1, m3, x[c + 3 * G]);
    }
    for (; c < m; c += G) cfma(a0, ldnt(Ar + (long long)c * lda), x[c]);
  }
  a0 = cadd(a0, a1);
  if (G == 1) return a0;
  red[t] = a0;
  __syncthreads();
  if (t < nr) {
    for (int k = 1; k < G; ++k) a0 = cadd(a0, red[k * nr + t]);
  }
  __syncthreads();
  return a0;
}

// Side s (0 left, 1 right, 2 bottom, 3 top) of the slot-th present side.
__device__ __forceinline__ int side_of_slot(int mask, int slot) {
  int seen = -1;
  for (int k = 0; k < 4; ++k)
    if ((mask >> k) & 1)
      if (++seen == slot) return k;
  return -1;
}

// Leaf upward pass (one block per leaf and column):
//   g = (alpha u0 + tau v0) / tau^2 on the interior nodes,
//   w = W g,  h = N_i w on the leaf's interface sides.
__global__ __launch_bounds__(kBlock) void k_leaf_up(LeafUpArgs a) {
  __shared__ double2 gs[kMaxQ2];
  __shared__ double2 ws[kMaxQ2];
  __shared__ double2 red[kBlock];
  const int leaf = blockIdx.x / a.ncol;
  const int col = blockIdx.x - leaf * a.ncol;
  const int pole = col / a.nrhs, rhs = col - pole * a.nrhs;
  const int q = a.q, q2 = q * q;
  const LeafDesc L = a.leaves[leaf];
  const PoleCoef pc = a.coef[pole];
  const double* x1 = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
  const double* x2 = x1 + a.n_int;
  const double* x3 = x2 + a.n_int;
  for (int t = threadIdx.x; t < q2; t += blockDim.x) {
    const double u1 = x1[t], u2 = x2[t], u3 = a.nsrc > 2 ? x3[t] : 0.0;
    gs[t] = make_double2(fma(pc.k1.x, u1, fma(pc.k2.x, u2, pc.k3.x * u3)),
                         fma(pc.k1.y, u1, fma(pc.k2.y, u2, pc.k3.y * u3)));
  }
  __syncthreads();
  const double2* W = a.ops + pole * a.pole_stride + L.op_off;
  const double2 acc = gemv_cm<kBlock>(W, q2, 0, q2, q2, gs, red);
  if (threadIdx.x < q2) {
    a.w[((long long)pole * a.w_pole + (long long)leaf * q2 + threadIdx.x) * a.nrhs + rhs] = acc;
    ws[threadIdx.x] = acc;
  }
  __syncthreads();
  double2* hout = a.h + ((long long)pole * a.h_pole + L.vec_off) * a.nrhs + rhs;
  for (int r = threadIdx.x; r < L.e; r += blockDim.x) {
    const int slot = r / q, t = r - slot * q;
    const int s = side_of_slot(L.side_mask, slot);
    const double* nr = a.nrow + ((s == 1 || s == 3) ? q : 0);
    const double sc = (s == 0) ? -a.sx : (s == 1) ? a.sx : (s == 2) ? -a.sy : a.sy;
    double2 sum = make_double2(0.0, 0.0);
    if (s < 2) {
      for (int k = 0; k < q; ++k) { sum.x += nr[k] * ws[k + q * t].x; sum.y += nr[k] * ws[k + q * t].y; }
    } else {
      for (int k = 0; k < q; ++k) { sum.x += nr[k] * ws[t + q * k].x; sum.y += nr[k] * ws[t + q * k].y; }
    }
    hout[(long long)r * a.nrhs] = make_double2(sc * sum.x, sc * sum.y);
  }
}

// Merge upward pass for one level (block = box, column, row block):
//   g3 = h_3^a + h_3^b,   h_par = [h_1^a; h_2^b] - Y g3.
__global__ __launch_bounds__(kBlock) void k_merge_up(MergeArgs a) {
  extern __shared__ double2 xs[];
  __shared__ double2 red[kBlock];
  const int per_box = a.ncol * a.row_blocks;
  const int box = blockIdx.x / per_box;
  const int rem = blockIdx.x - box * per_box;
  const int col = rem / a.row_blocks, rb = rem - col * a.row_blocks;
  const int pole = col / a.nrhs, rhs = col - pole * a.nrhs;
  const int R = a.nrhs;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  const int r0 = rb * kBlock;
  if (r0 >= ext && !(rb == 0 && ext == 0)) return;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const double2* hc = a.child + (long long)pole * a.child_pole * R + rhs;
  for (int t = threadIdx.x; t < n3; t += blockDim.x)
    xs[t] = cadd(hc[(long long)(B.a_vec + i3a[t]) * R], hc[(long long)(B.b_vec + i3b[t]) * R]);
  __syncthreads();
  if (rb == 0) {
    double2* g3 = a.g3 + ((long long)pole * a.g3_pole + B.g3_off) * R + rhs;
    for (int t = threadIdx.x; t < n3; t += blockDim.x) g3[(long long)t * R] = xs[t];
  }
  if (ext == 0) return;
  const int nr = min(ext - r0, kBlock);
  const double2* Y = a.ops + pole * a.pole_stride + B.op_off + (long long)n3 * (ext + n3);
  const double2 acc = gemv_cm<kBlock>(Y, ext, r0, nr, n3, xs, red);
  const int r = r0 + threadIdx.x;
  if (threadIdx.x < nr) {
    const double2 base = (r < n1) ? hc[(long long)(B.a_vec + i1[r]) * R] : hc[(long long)(B.b_vec + i2[r - n1]) * R];
    a.self[((long long)pole * a.self_pole + B.vec_off + r) * R + rhs] = make_double2(base.x - acc.x, base.y - acc.y);
  }
}

// Merge downward pass for one level (block = box, column, row block):
//   u3 = -Z [u_ext; g3], scattered with u_ext into the children's vectors.
__global__ __launch_bounds__(kBlock) void k_merge_down(MergeArgs a) {
  extern __shared__ double2 xs[];
  __shared__ double2 red[kBlock];
  const int per_box = a.ncol * a.row_blocks;
  const int box = blockIdx.x / per_box;
  const int rem = blockIdx.x - box * per_box;
  const int col = rem / a.row_blocks, rb = rem - col * a.row_blocks;
  const int pole = col / a.nrhs, rhs = col - pole * a.nrhs;
  const int R = a.nrhs;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  const int r0 = rb * kBlock;
  if (r0 >= n3) return;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const double2* up = a.self + ((long long)pole * a.self_pole + B.vec_off) * R + rhs;
  const double2* g3 = a.g3 + ((long long)pole * a.g3_pole + B.g3_off) * R + rhs;
  for (int t = threadIdx.x; t < ext; t += blockDim.x) xs[t] = up[(long long)t * R];
  for (int t = threadIdx.x; t < n3; t += blockDim.x) xs[ext + t] = g3[(long long)t * R];
  __syncthreads();
  double2* uc = a.child + (long long)pole * a.child_pole * R + rhs;
  if (rb == 0) {
    for (int k = threadIdx.x; k < n1; k += blockDim.x) uc[(long long)(B.a_vec + i1[k]) * R] = xs[k];
    for (int k = threadIdx.x; k < n2; k += blockDim.x) uc[(long long)(B.b_vec + i2[k]) * R] = xs[n1 + k];
  }
  const int nr = min(n3 - r0, kBlock);
  const double2* Z = a.ops + pole * a.pole_stride + B.op_off;
  const double2 acc = gemv_cm<kBlock>(Z, n3, r0, nr, ext + n3, xs, red);
  if (threadIdx.x < nr) {
    const int r = r0 + threadIdx.x;
    const double2 u3 = make_double2(-acc.x, -acc.y);
    uc[(long long)(B.a_vec + i3a[r]) * R] = u3;
    uc[(long long)(B.b_vec + i3b[r]) * R] = u3;
  }
}

// Leaf downward pass (block = leaf, column): y = w - S u_e, in place of w.
__global__ __launch_bounds__(kBlock) void k_leaf_down(LeafDownArgs a) {
  __shared__ double2 us[4 * (kMaxP - 2)];
  __shared__ double2 red[kBlock];
  const int leaf = blockIdx.x / a.ncol;
  const int col = blockIdx.x - leaf * a.ncol;
  const int pole = col / a.nrhs, rhs = col - pole * a.nrhs;
  const int R = a.nrhs;
  const int q2 = a.q * a.q;
  const LeafDesc L = a.leaves[leaf];
  const double2* ue = a.u + ((long long)pole * a.u_pole + L.vec_off) * R + rhs;
  for (int c = threadIdx.x; c < L.e; c += blockDim.x) us[c] = ue[(long long)c * R];
  __syncthreads();
  const double2* S = a.ops + pole * a.pole_stride + L.op_off + (long long)q2 * q2;
  const double2 acc = gemv_cm<kBlock>(S, q2, 0, q2, L.e, us, red);
  if (threadIdx.x < q2) {
    double2* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2 + threadIdx.x) * R + rhs;
    const double2 wt = *w;
    *w = make_double2(wt.x - acc.x, wt.y - acc.y);
  }
}

// Pole sum and post-map (block = leaf, rhs), FP64, fixed pole order:
//   u' = sum_m Re(cu_m y_m),  v' = (beta u0 + sum_m Re(cv_m y_m)) / tau.
__global__ __launch_bounds__(kBlock) void k_pole_sum(PoleSumArgs a) {
  const int leaf = blockIdx.x / a.nrhs;
  const int rhs = blockIdx.x - leaf * a.nrhs;
  const int q2 = a.q * a.q;
  const LeafDesc L = a.leaves[leaf];
  double* u = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
  double* v = u + a.n_int;
  for (int t = threadIdx.x; t < q2; t += blockDim.x) {
    double su = 0.0, sv = 0.0;
    for (int pole = 0; pole < a.npole; ++pole) {
      const double2 y = a.y[((long long)pole * a.y_pole + (long long)leaf * q2 + t) * a.nrhs + rhs];
      const PoleCoef c = a.coef[pole];
      su = fma(c.cu.x, y.x, fma(-c.cu.y, y.y, su));
      sv = fma(c.cv.x, y.x, fma(-c.cv.y, y.y, sv));
    }
    const double u0 = u[t];
    u[t] = su;
    v[t] = fma(a.beta, u0, sv) * a.inv_tau;
  }
}

// ---- launchers -------------------------------------------------------------

hipError_t launch_leaf_up(const LeafUpArgs& a, int n_leaf, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_up, dim3(n_leaf * a.ncol), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_merge_up(const MergeArgs& a, int n_box, int max_n3, hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)(max_n3 > 0 ? max_n3 : 1);
  hipLaunchKernelGGL(k_merge_up, dim3(n_box * a.ncol * a.row_blocks), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_merge_down(const MergeArgs& a, int n_box, int max_x, hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)(max_x > 0 ? max_x : 1);
  hipLaunchKernelGGL(k_merge_down, dim3(n_box * a.ncol * a.row_blocks), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_leaf_down(const LeafDownArgs& a, int n_leaf, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_down, dim3(n_leaf * a.ncol), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pole_sum(const PoleSumArgs& a, int n_leaf, hipStream_t s) {
  hipLaunchKernelGGL(k_pole_sum, dim3(n_leaf * a.nrhs), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace hx
