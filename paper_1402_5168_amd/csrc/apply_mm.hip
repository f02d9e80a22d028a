// Solve-stage sweeps for many right-hand sides at once on the matrix cores.
//
// With r right-hand sides every stored operator entry is used r times per
// step, so each sweep becomes a batch of small complex GEMMs
//     C (rows x RT) = A (rows x m, column-major, HBM) * B (m x RT, LDS),
// RT = 16 or 32 right-hand sides per block.  A complex product is four real
// MFMAs (v_mfma_*_16x16x4) into four accumulators (re*re, im*im, re*im,
// im*re) combined at the end.  A wave owns one 16-row tile; it loads each
// A entry exactly once (16 consecutive rows of 4 columns per instruction)
// and reads its B fragment from LDS, where B is staged in k-chunks by the
// whole block.  Vectors are stored [pole][node][rhs] (rhs fastest), so the
// B gathers and the C stores of 16 consecutive right-hand sides are
// contiguous.
#include "hx_kernels.h"

namespace hx {

template <class T> struct MM;
template <> struct MM<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  typedef double2 C;
  __device__ static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // D[i][j] of the 16x16 result sits in lane j + 16*(i%4), register i/4
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct MM<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  typedef float2 C;
  __device__ static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // D[i][j] sits in lane j + 16*(i/4), register i%4
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v2f_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const v2d_t v = __builtin_nontemporal_load(reinterpret_cast<const v2d_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const v2f_t v = __builtin_nontemporal_load(reinterpret_cast<const v2f_t*>(p));
  return make_float2(v.x, v.y);
}

template <class T, int NT>
struct Acc {
  typename MM<T>::v4 rr[NT], ii[NT], ri[NT], ir[NT];
  __device__ void zero() {
    for (int t = 0; t < NT; ++t)
      for (int v = 0; v < 4; ++v) rr[t][v] = ii[t][v] = ri[t][v] = ir[t][v] = T(0);
  }
};

// One wave: acc += A[its 16-row tile, columns k_lo .. k_lo+kc) * Bs[0..kc).
// A points at row 0 of the operator; rows >= nrows and columns >= kc give 0
// (no load is issued for them).  Bs holds kc rows rounded up to a multiple
// of 4, zero-padded, with row stride bst.
template <class T, int NT>
__device__ __forceinline__ void mm_chunk(Acc<T, NT>& acc, const typename MM<T>::C* __restrict__ A,
                                         long long lda, int row0, int nrows, int k_lo, int kc,
                                         const typename MM<T>::C* __restrict__ Bs, int bst) {
  using C = typename MM<T>::C;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kk = lane >> 4;
  const bool rv = row0 + i < nrows;
  const C* Ar = A + row0 + i + (long long)k_lo * lda;
  const int kcp = (kc + 3) & ~3;
  int k4 = 0;
  for (; k4 + 8 <= kcp; k4 += 8) {
    const int k0 = k4 + kk, k1 = k4 + 4 + kk;
    C a0, a1;
    a0.x = a0.y = a1.x = a1.y = T(0);
    if (rv && k0 < kc) a0 = ld_stream(Ar + (long long)k0 * lda);
    if (rv && k1 < kc) a1 = ld_stream(Ar + (long long)k1 * lda);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const C b0 = Bs[k0 * bst + t * 16 + i];
      acc.rr[t] = MM<T>::mma(a0.x, b0.x, acc.rr[t]);
      acc.ii[t] = MM<T>::mma(a0.y, b0.y, acc.ii[t]);
      acc.ri[t] = MM<T>::mma(a0.x, b0.y, acc.ri[t]);
      acc.ir[t] = MM<T>::mma(a0.y, b0.x, acc.ir[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const C b1 = Bs[k1 * bst + t * 16 + i];
      acc.rr[t] = MM<T>::mma(a1.x, b1.x, acc.rr[t]);
      acc.ii[t] = MM<T>::mma(a1.y, b1.y, acc.ii[t]);
      acc.ri[t] = MM<T>::mma(a1.x, b1.y, acc.ri[t]);
      acc.ir[t] = MM<T>::mma(a1.y, b1.x, acc.ir[t]);
    }
  }
  for (; k4 < kcp; k4 += 4) {
    const int k = k4 + kk;
    C a;
    a.x = a.y = T(0);
    if (rv && k < kc) a = ld_stream(Ar + (long long)k * lda);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const C b = Bs[k * bst + t * 16 + i];
      acc.rr[t] = MM<T>::mma(a.x, b.x, acc.rr[t]);
      acc.ii[t] = MM<T>::mma(a.y, b.y, acc.ii[t]);
      acc.ri[t] = MM<T>::mma(a.x, b.y, acc.ri[t]);
      acc.ir[t] = MM<T>::mma(a.y, b.x, acc.ir[t]);
    }
  }
}

// Visit the wave's results: f(row, j, value) for row < nrows, j < RT.
template <class T, int NT, class F>
__device__ __forceinline__ void mm_emit(const Acc<T, NT>& acc, int row0, int nrows, F&& f) {
  using C = typename MM<T>::C;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + MM<T>::row(lane, v);
      if (row < nrows) {
        C c;
        c.x = acc.rr[t][v] - acc.ii[t][v];
        c.y = acc.ri[t][v] + acc.ir[t][v];
        f(row, t * 16 + (lane & 15), c);
      }
    }
}

constexpr int kKC = 64;  // k-chunk of B staged in LDS

// ---- leaf upward: g from the state, w = W g, h = N_i w ------------------------
// block = (leaf, pole, rhs tile); every row tile of W is handled by the block.
template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_up_mm(MmLeafUpArgs<T> a) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  extern __shared__ unsigned char smem[];
  C* gs = reinterpret_cast<C*>(smem);
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const int rt = blockIdx.x % n_rt;
  const int lp = blockIdx.x / n_rt;
  const int pole = lp % a.npole, leaf = lp / a.npole;
  const int q = a.q, q2 = q * q, q2p = (q2 + 3) & ~3;
  const LeafDesc L = a.leaves[leaf];
  const double2 al = a.coef[pole].alpha;
  const int r = a.nrhs;
  for (int idx = threadIdx.x; idx < q2p * RT; idx += blockDim.x) {
    const int j = idx / q2p, k = idx - j * q2p;
    const int rhs = rt * RT + j;
    C g;
    g.x = g.y = T(0);
    if (k < q2 && rhs < r) {
      const double* u0 = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
      const double uu = u0[k], vv = u0[a.n_int + k];
      g.x = T(fma(al.x * a.inv_tau2, uu, vv * a.inv_tau));
      g.y = T(al.y * a.inv_tau2 * uu);
    }
    gs[k * BST + j] = g;
  }
  __syncthreads();
  const C* W = a.ops + pole * a.pole_stride + L.op_off;
  C* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
  const int wave = threadIdx.x >> 6;
  for (int tile = wave; tile * 16 < q2; tile += kBlock / 64) {
    Acc<T, NT> acc;
    acc.zero();
    mm_chunk<T, NT>(acc, W, q2, tile * 16, q2, 0, q2, gs, BST);
    mm_emit<T, NT>(acc, tile * 16, q2, [&](int row, int j, C c) {
      const int rhs = rt * RT + j;
      if (rhs < r) w[(long long)row * r + rhs] = c;
    });
  }
  __syncthreads();
  C* h = a.h + ((long long)pole * a.h_pole + L.vec_off) * r;
  for (int idx = threadIdx.x; idx < L.e * RT; idx += blockDim.x) {
    const int re = idx / RT, j = idx - re * RT;
    const int rhs = rt * RT + j;
    if (rhs >= r) continue;
    const int slot = re / q, t = re - slot * q;
    int s = -1, seen = -1;
    for (int k = 0; k < 4; ++k)
      if ((L.side_mask >> k) & 1)
        if (++seen == slot) { s = k; break; }
    const double* nr = a.nrow + ((s == 1 || s == 3) ? q : 0);
    const double sc = (s == 0) ? -a.sx : (s == 1) ? a.sx : (s == 2) ? -a.sy : a.sy;
    T sx_ = T(0), sy_ = T(0);
    for (int k = 0; k < q; ++k) {
      const int node = (s < 2) ? (k + q * t) : (t + q * k);
      const C wv = w[(long long)node * r + rhs];
      sx_ += T(nr[k]) * wv.x;
      sy_ += T(nr[k]) * wv.y;
    }
    C hv;
    hv.x = T(sc) * sx_;
    hv.y = T(sc) * sy_;
    h[(long long)re * r + rhs] = hv;
  }
}

// ---- merge upward: g3 = h3a + h3b (- j3), h_par = [h1a; h2b] - Y g3 ----------
// block = (box, pole, rhs tile, row group of 64 rows of Y)
template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_merge_up_mm(MmMergeArgs<T> a) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[kKC * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = blockIdx.x;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int box = rest / a.npole;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  if (rg > 0 && rg * 64 >= ext) return;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const int r = a.nrhs;
  const C* hc = a.child + (long long)pole * a.child_pole * r;
  C* g3 = a.g3 + ((long long)pole * a.g3_pole + B.g3_off) * r;
  const C* Y = a.ops + pole * a.pole_stride + B.op_off + (long long)n3 * (ext + n3);
  const int row0 = rg * 64 + (threadIdx.x >> 6) * 16;
  Acc<T, NT> acc;
  acc.zero();
  for (int k0 = 0; k0 < n3; k0 += kKC) {
    const int kc = min(kKC, n3 - k0), kcp = (kc + 3) & ~3;
    for (int idx = threadIdx.x; idx < kcp * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = rt * RT + j;
      C v;
      v.x = v.y = T(0);
      if (k < kc && rhs < r) {
        const C x = hc[(long long)(B.a_vec + i3a[k0 + k]) * r + rhs];
        const C y = hc[(long long)(B.b_vec + i3b[k0 + k]) * r + rhs];
        v.x = x.x + y.x;
        v.y = x.y + y.y;
        if (rg == 0) g3[(long long)(k0 + k) * r + rhs] = v;
      }
      Bs[k * BST + j] = v;
    }
    __syncthreads();
    if (row0 < ext) mm_chunk<T, NT>(acc, Y, ext, row0, ext, k0, kc, Bs, BST);
    __syncthreads();
  }
  if (row0 >= ext) return;
  C* hp = a.self + ((long long)pole * a.self_pole + B.vec_off) * r;
  mm_emit<T, NT>(acc, row0, ext, [&](int row, int j, C c) {
    const int rhs = rt * RT + j;
    if (rhs >= r) return;
    const C base = (row < n1) ? hc[(long long)(B.a_vec + i1[row]) * r + rhs]
                              : hc[(long long)(B.b_vec + i2[row - n1]) * r + rhs];
    C o;
    o.x = base.x - c.x;
    o.y = base.y - c.y;
    hp[(long long)row * r + rhs] = o;
  });
}

// ---- merge downward: u3 = -Z [u_ext; g3], scattered to the children --------
template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_merge_down_mm(MmMergeArgs<T> a) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[kKC * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = blockIdx.x;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int box = rest / a.npole;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2, m = ext + n3;
  if (rg * 64 >= n3) return;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const int r = a.nrhs;
  const C* up = a.self + ((long long)pole * a.self_pole + B.vec_off) * r;
  const C* g3 = a.g3 + ((long long)pole * a.g3_pole + B.g3_off) * r;
  C* uc = a.child + (long long)pole * a.child_pole * r;
  if (rg == 0) {
    for (int idx = threadIdx.x; idx < ext * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = rt * RT + j;
      if (rhs >= r) continue;
      const C v = up[(long long)k * r + rhs];
      if (k < n1) uc[(long long)(B.a_vec + i1[k]) * r + rhs] = v;
      else uc[(long long)(B.b_vec + i2[k - n1]) * r + rhs] = v;
    }
  }
  const C* Z = a.ops + pole * a.pole_stride + B.op_off;
  const int row0 = rg * 64 + (threadIdx.x >> 6) * 16;
  Acc<T, NT> acc;
  acc.zero();
  for (int k0 = 0; k0 < m; k0 += kKC) {
    const int kc = min(kKC, m - k0), kcp = (kc + 3) & ~3;
    for (int idx = threadIdx.x; idx < kcp * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = rt * RT + j;
      C v;
      v.x = v.y = T(0);
      if (k < kc && rhs < r) {
        const int kg = k0 + k;
        v = (kg < ext) ? up[(long long)kg * r + rhs] : g3[(long long)(kg - ext) * r + rhs];
      }
      Bs[k * BST + j] = v;
    }
    __syncthreads();
    if (row0 < n3) mm_chunk<T, NT>(acc, Z, n3, row0, n3, k0, kc, Bs, BST);
    __syncthreads();
  }
  if (row0 >= n3) return;
  mm_emit<T, NT>(acc, row0, n3, [&](int row, int j, C c) {
    const int rhs = rt * RT + j;
    if (rhs >= r) return;
    C u3;
    u3.x = -c.x;
    u3.y = -c.y;
    uc[(long long)(B.a_vec + i3a[row]) * r + rhs] = u3;
    uc[(long long)(B.b_vec + i3b[row]) * r + rhs] = u3;
  });
}

// ---- leaf downward: y = w - S u_e (in place of w) -----------------------------
template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_down_mm(MmLeafDownArgs<T> a) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[4 * (kMaxP - 2) * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = blockIdx.x;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int leaf = rest / a.npole;
  const int q2 = a.q * a.q;
  if (rg * 64 >= q2) return;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs, e = L.e, ep = (e + 3) & ~3;
  const C* ue = a.u + ((long long)pole * a.u_pole + L.vec_off) * r;
  for (int idx = threadIdx.x; idx < ep * RT; idx += blockDim.x) {
    const int k = idx / RT, j = idx - k * RT;
    const int rhs = rt * RT + j;
    C v;
    v.x = v.y = T(0);
    if (k < e && rhs < r) v = ue[(long long)k * r + rhs];
    Bs[k * BST + j] = v;
  }
  __syncthreads();
  const int row0 = rg * 64 + (threadIdx.x >> 6) * 16;
  if (row0 >= q2) return;
  const C* S = a.ops + pole * a.pole_stride + L.op_off + (long long)q2 * q2;
  Acc<T, NT> acc;
  acc.zero();
  if (e > 0) mm_chunk<T, NT>(acc, S, q2, row0, q2, 0, e, Bs, BST);
  C* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
  mm_emit<T, NT>(acc, row0, q2, [&](int row, int j, C c) {
    const int rhs = rt * RT + j;
    if (rhs >= r) return;
    C& y = w[(long long)row * r + rhs];
    C o = y;
    o.x -= c.x;
    o.y -= c.y;
    y = o;
  });
}

// ---- leaf downward fused with the pole sum ----------------------------------------
// block = (leaf, rhs tile, row group); it walks the poles in order:
//   y_m = w_m - S_m u_e,m,  u' = sum_m Re(cu_m y_m),  v' = (beta u0 + sum_m Re(cv_m y_m)) / tau,
// so the per-pole solutions never go back to HBM.  Accumulation is FP64.
template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_down_sum_mm(MmLeafDownArgs<T> a) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[4 * (kMaxP - 2) * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = blockIdx.x;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt;
  const int leaf = rest / n_rt;
  const int q2 = a.q * a.q;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs, e = L.e, ep = (e + 3) & ~3;
  const int row0 = rg * 64 + (threadIdx.x >> 6) * 16;
  const int lane = threadIdx.x & 63;
  double su[NT][4], sv[NT][4];
  for (int t = 0; t < NT; ++t)
    for (int v = 0; v < 4; ++v) su[t][v] = sv[t][v] = 0.0;
  for (int pole = 0; pole < a.npole; ++pole) {
    const C* ue = a.u + ((long long)pole * a.u_pole + L.vec_off) * r;
    for (int idx = threadIdx.x; idx < ep * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = rt * RT + j;
      C v;
      v.x = v.y = T(0);
      if (k < e && rhs < r) v = ue[(long long)k * r + rhs];
      Bs[k * BST + j] = v;
    }
    __syncthreads();
    if (row0 < q2) {
      const C* S = a.ops + pole * a.pole_stride + L.op_off + (long long)q2 * q2;
      Acc<T, NT> acc;
      acc.zero();
      if (e > 0) mm_chunk<T, NT>(acc, S, q2, row0, q2, 0, e, Bs, BST);
      const C* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
      const PoleCoef pc = a.coef[pole];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + MM<T>::row(lane, v);
          const int rhs = rt * RT + t * 16 + (lane & 15);
          if (row < q2 && rhs < r) {
            const C wv = w[(long long)row * r + rhs];
            const double yr = double(wv.x) - double(acc.rr[t][v] - acc.ii[t][v]);
            const double yi = double(wv.y) - double(acc.ri[t][v] + acc.ir[t][v]);
            su[t][v] = fma(pc.cu.x, yr, fma(-pc.cu.y, yi, su[t][v]));
            sv[t][v] = fma(pc.cv.x, yr, fma(-pc.cv.y, yi, sv[t][v]));
          }
        }
    }
    __syncthreads();
  }
  if (row0 >= q2) return;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + MM<T>::row(lane, v);
      const int rhs = rt * RT + t * 16 + (lane & 15);
      if (row < q2 && rhs < r) {
        double* u = a.state + rhs * a.rhs_stride + (long long)L.elem * q2 + row;
        const double u0 = u[0];
        u[0] = su[t][v];
        u[a.n_int] = fma(a.beta, u0, sv[t][v]) * a.inv_tau;
      }
    }
}

// ---- launchers -----------------------------------------------------------------

template <class T, int NT>
size_t leaf_up_lds(int q) {
  return sizeof(typename MM<T>::C) * (size_t)((q * q + 3) & ~3) * (16 * NT + 1);
}

template <class T, int NT>
static hipError_t leaf_up_t(const MmLeafUpArgs<T>& a, int n_leaf, hipStream_t s) {
  constexpr int RT = 16 * NT;
  const size_t lds = leaf_up_lds<T, NT>(a.q);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leaf_up_mm<T, NT>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int n_rt = (a.nrhs + RT - 1) / RT;
  hipLaunchKernelGGL((k_leaf_up_mm<T, NT>), dim3(n_leaf * a.npole * n_rt), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

// Two tiles of 16 right-hand sides per block when the staged right-hand
// sides fit in 64 KiB of LDS, otherwise one (more blocks, W read per tile).
template <class T>
hipError_t launch_leaf_up_mm(const MmLeafUpArgs<T>& a, int n_leaf, int nt, hipStream_t s) {
  if (nt == 2 && leaf_up_lds<T, 2>(a.q) <= 65536) return leaf_up_t<T, 2>(a, n_leaf, s);
  return leaf_up_t<T, 1>(a, n_leaf, s);
}

template <class T>
hipError_t launch_merge_up_mm(const MmMergeArgs<T>& a, int n_box, int nt, hipStream_t s) {
  const int RT = 16 * nt;
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const dim3 grid(n_box * a.npole * n_rt * a.row_groups);
  if (nt == 2) hipLaunchKernelGGL((k_merge_up_mm<T, 2>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_merge_up_mm<T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_merge_down_mm(const MmMergeArgs<T>& a, int n_box, int nt, hipStream_t s) {
  const int RT = 16 * nt;
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const dim3 grid(n_box * a.npole * n_rt * a.row_groups);
  if (nt == 2) hipLaunchKernelGGL((k_merge_down_mm<T, 2>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_merge_down_mm<T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_leaf_down_mm(const MmLeafDownArgs<T>& a, int n_leaf, int nt, hipStream_t s) {
  const int RT = 16 * nt;
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const dim3 grid(n_leaf * a.npole * n_rt * a.row_groups);
  if (nt == 2) hipLaunchKernelGGL((k_leaf_down_mm<T, 2>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_leaf_down_mm<T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_leaf_down_sum_mm(const MmLeafDownArgs<T>& a, int n_leaf, int nt, hipStream_t s) {
  const int RT = 16 * nt;
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const dim3 grid(n_leaf * n_rt * a.row_groups);
  if (nt == 2) hipLaunchKernelGGL((k_leaf_down_sum_mm<T, 2>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_leaf_down_sum_mm<T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_leaf_down_sum_mm<double>(const MmLeafDownArgs<double>&, int, int, hipStream_t);
template hipError_t launch_leaf_up_mm<double>(const MmLeafUpArgs<double>&, int, int, hipStream_t);
template hipError_t launch_merge_up_mm<double>(const MmMergeArgs<double>&, int, int, hipStream_t);
template hipError_t launch_merge_down_mm<double>(const MmMergeArgs<double>&, int, int, hipStream_t);
template hipError_t launch_leaf_down_mm<double>(const MmLeafDownArgs<double>&, int, int, hipStream_t);

}  // namespace hx
