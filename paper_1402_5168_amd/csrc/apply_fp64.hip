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

// acc += A[row + k*lda] * x[k], k = 0..n-1, with four loads in flight.
__device__ __forceinline__ double2 col_dot(const double2* __restrict__ A, long long lda,
                                           const double2* __restrict__ x, int n) {
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    const double2 m0 = ldnt(A + (k + 0) * lda);
    const double2 m1 = ldnt(A + (k + 1) * lda);
    const double2 m2 = ldnt(A + (k + 2) * lda);
    const double2 m3 = ldnt(A + (k + 3) * lda);
    cfma(a0, m0, x[k + 0]);
    cfma(a1, m1, x[k + 1]);
    cfma(a0, m2, x[k + 2]);
    cfma(a1, m3, x[k + 3]);
  }
  for (; k < n; ++k) cfma(a0, ldnt(A + k * lda), x[k]);
  return cadd(a0, a1);
}

// Leaf upward pass (one block per leaf and column):
//   g = (alpha u0 + tau v0) / tau^2 on the interior nodes,
//   w = W g,  h = N_i w on the leaf's interface sides.
__global__ __launch_bounds__(kBlock) void k_leaf_up(LeafUpArgs a) {
  __shared__ double2 gs[kMaxQ2];
  __shared__ double2 ws[kMaxQ2];
  const int leaf = blockIdx.x / a.ncol;
  const int col = blockIdx.x - leaf * a.ncol;
  const int pole = col / a.nrhs, rhs = col - pole * a.nrhs;
  const int q = a.q, q2 = q * q;
  const LeafDesc L = a.leaves[leaf];
  const double2 al = a.coef[pole].alpha;
  const double* u0 = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
  const double* v0 = u0 + a.n_int;
  for (int t = threadIdx.x; t < q2; t += blockDim.x) {
    const double uu = u0[t], vv = v0[t];
    gs[t] = make_double2(fma(al.x * a.inv_tau2, uu, vv * a.inv_tau), al.y * a.inv_tau2 * uu);
  }
  __syncthreads();
  const double2* W = a.ops + pole * a.pole_stride + L.op_off;
  double2* wout = a.w + col * a.w_col_stride + (long long)leaf * q2;
  for (int t = threadIdx.x; t < q2; t += blockDim.x) {
    const double2 acc = col_dot(W + t, q2, gs, q2);
    wout[t] = acc;
    ws[t] = acc;
  }
  __syncthreads();
  double2* hout = a.h + col * a.h_col_stride + L.vec_off;
  for (int r = threadIdx.x; r < L.e; r += blockDim.x) {
    const int slot = r / q, t = r - slot * q;
    int s = -1, seen = -1;
    for (int k = 0; k < 4; ++k)
      if ((L.side_mask >> k) & 1)
        if (++seen == slot) { s = k; break; }
    const double* nr = a.nrow + ((s == 1 || s == 3) ? q : 0);
    const double sc = (s == 0) ? -a.sx : (s == 1) ? a.sx : (s == 2) ? -a.sy : a.sy;
    double2 sum = make_double2(0.0, 0.0);
    if (s < 2) {
      for (int k = 0; k < q; ++k) { sum.x += nr[k] * ws[k + q * t].x; sum.y += nr[k] * ws[k + q * t].y; }
    } else {
      for (int k = 0; k < q; ++k) { sum.x += nr[k] * ws[t + q * k].x; sum.y += nr[k] * ws[t + q * k].y; }
    }
    hout[r] = make_double2(sc * sum.x, sc * sum.y);
  }
}

// Merge upward pass for one level (block = box, column, row block):
//   g3 = h_3^a + h_3^b,   h_par = [h_1^a; h_2^b] - Y g3.
__global__ __launch_bounds__(kBlock) void k_merge_up(MergeArgs a) {
  extern __shared__ double2 xs[];
  const int per_box = a.ncol * a.row_blocks;
  const int box = blockIdx.x / per_box;
  const int rem = blockIdx.x - box * per_box;
  const int col = rem / a.row_blocks, rb = rem - col * a.row_blocks;
  const int pole = col / a.nrhs;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const double2* hc = a.child + col * a.child_col_stride;
  for (int t = threadIdx.x; t < n3; t += blockDim.x)
    xs[t] = cadd(hc[B.a_vec + i3a[t]], hc[B.b_vec + i3b[t]]);
  __syncthreads();
  if (rb == 0) {
    double2* g3 = a.g3 + col * a.g3_col_stride + B.g3_off;
    for (int t = threadIdx.x; t < n3; t += blockDim.x) g3[t] = xs[t];
  }
  const int r = rb * blockDim.x + threadIdx.x;
  if (r >= ext) return;
  const double2* Y = a.ops + pole * a.pole_stride + B.op_off + (long long)n3 * (ext + n3);
  const double2 acc = col_dot(Y + r, ext, xs, n3);
  const double2 base = (r < n1) ? hc[B.a_vec + i1[r]] : hc[B.b_vec + i2[r - n1]];
  a.self[col * a.self_col_stride + B.vec_off + r] = make_double2(base.x - acc.x, base.y - acc.y);
}

// Merge downward pass for one level (block = box, column, row block):
//   u3 = -Z [u_ext; g3], scattered with u_ext into the children's vectors.
__global__ __launch_bounds__(kBlock) void k_merge_down(MergeArgs a) {
  extern __shared__ double2 xs[];
  const int per_box = a.ncol * a.row_blocks;
  const int box = blockIdx.x / per_box;
  const int rem = blockIdx.x - box * per_box;
  const int col = rem / a.row_blocks, rb = rem - col * a.row_blocks;
  const int pole = col / a.nrhs;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const double2* up = a.self + col * a.self_col_stride + B.vec_off;
  const double2* g3 = a.g3 + col * a.g3_col_stride + B.g3_off;
  for (int t = threadIdx.x; t < ext; t += blockDim.x) xs[t] = up[t];
  for (int t = threadIdx.x; t < n3; t += blockDim.x) xs[ext + t] = g3[t];
  __syncthreads();
  double2* uc = a.child + col * a.child_col_stride;
  if (rb == 0) {
    for (int k = threadIdx.x; k < n1; k += blockDim.x) uc[B.a_vec + i1[k]] = xs[k];
    for (int k = threadIdx.x; k < n2; k += blockDim.x) uc[B.b_vec + i2[k]] = xs[n1 + k];
  }
  const int r = rb * blockDim.x + threadIdx.x;
  if (r >= n3) return;
  const double2* Z = a.ops + pole * a.pole_stride + B.op_off;
  const double2 acc = col_dot(Z + r, n3, xs, ext + n3);
  const double2 u3 = make_double2(-acc.x, -acc.y);
  uc[B.a_vec + i3a[r]] = u3;
  uc[B.b_vec + i3b[r]] = u3;
}

// Leaf downward pass (block = leaf, column): y = w - S u_e, in place of w.
__global__ __launch_bounds__(kBlock) void k_leaf_down(LeafDownArgs a) {
  __shared__ double2 us[4 * (kMaxP - 2)];
  const int leaf = blockIdx.x / a.ncol;
  const int col = blockIdx.x - leaf * a.ncol;
  const int pole = col / a.nrhs;
  const int q2 = a.q * a.q;
  const LeafDesc L = a.leaves[leaf];
  const double2* ue = a.u + col * a.u_col_stride + L.vec_off;
  for (int c = threadIdx.x; c < L.e; c += blockDim.x) us[c] = ue[c];
  __syncthreads();
  const double2* S = a.ops + pole * a.pole_stride + L.op_off + (long long)q2 * q2;
  double2* w = a.w + col * a.w_col_stride + (long long)leaf * q2;
  for (int t = threadIdx.x; t < q2; t += blockDim.x) {
    const double2 acc = col_dot(S + t, q2, us, L.e);
    const double2 wt = w[t];
    w[t] = make_double2(wt.x - acc.x, wt.y - acc.y);
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
      const int col = pole * a.nrhs + rhs;
      const double2 y = a.y[col * a.y_col_stride + (long long)leaf * q2 + t];
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
