// Solve-stage sweeps for many right-hand sides at once on the matrix cores.
//
// With r right-hand sides every stored operator entry is used r times per
// step, so each sweep becomes a batch of small complex GEMMs
//     C (rows x RT) = A (rows x m, column-major, HBM) * B (m x RT, LDS),
// RT = 16 or 32 right-hand sides per block.  A complex product is four real
// MFMAs (v_mfma_*_16x16x4) into two accumulators, the real and the
// imaginary part.  A wave owns one 16-row tile; it streams each A entry
// exactly once (16 consecutive rows of 4 columns per load) and reads its B
// fragment from LDS, where B is staged in k-chunks by the whole block.  Vectors are stored [pole][node][rhs] (rhs fastest), so the
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

// Accumulators of one wave's 16-row tile.  FP32 tiles also keep FP64
// running sums: the MFMA accumulates a group of k-steps in FP32, then
// flush() adds the group into FP64, so the rounding error does not grow
// with the depth of long products (merge operators reach k ~ 10^3).
template <class T, int NT>
struct Acc {
  static constexpr bool kWide = sizeof(T) == sizeof(float);
  typedef double d4 __attribute__((ext_vector_type(4)));
  typename MM<T>::v4 re[NT], im[NT];
  d4 re64[NT], im64[NT];
  __device__ void zero() {
    for (int t = 0; t < NT; ++t)
      for (int v = 0; v < 4; ++v) {
        re[t][v] = im[t][v] = T(0);
        re64[t][v] = im64[t][v] = 0.0;
      }
  }
  __device__ void flush() {
    if constexpr (kWide) {
      for (int t = 0; t < NT; ++t)
        for (int v = 0; v < 4; ++v) {
          re64[t][v] += double(re[t][v]);
          im64[t][v] += double(im[t][v]);
          re[t][v] = im[t][v] = T(0);
        }
    }
  }
  __device__ double vre(int t, int v) const {
    if constexpr (kWide) return re64[t][v] + double(re[t][v]);
    else return re[t][v];
  }
  __device__ double vim(int t, int v) const {
    if constexpr (kWide) return im64[t][v] + double(im[t][v]);
    else return im[t][v];
  }
};

// One complex k-step of 4 columns on a 16-row tile: acc += a * Bk.  The
// first half-products of every column tile are issued before the second
// halves, so that MFMAs into the same accumulator sit further apart.
template <class T, int NT>
__device__ __forceinline__ void mma_step(Acc<T, NT>& acc, const typename MM<T>::C a,
                                         const typename MM<T>::C* __restrict__ Bk) {
  using C = typename MM<T>::C;
  const int i = threadIdx.x & 15;
  const T nay = -a.y;
  C b[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) b[t] = Bk[t * 16 + i];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc.re[t] = MM<T>::mma(a.x, b[t].x, acc.re[t]);
    acc.im[t] = MM<T>::mma(a.x, b[t].y, acc.im[t]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc.re[t] = MM<T>::mma(nay, b[t].y, acc.re[t]);
    acc.im[t] = MM<T>::mma(a.y, b[t].x, acc.im[t]);
  }
}

// The A loads of one product chunk.  mm_prime issues the first PF k-steps'
// loads; a caller may prime before it stages B, so that their latency
// overlaps the staging, then mm_run consumes them.  The loads go through a
// buffer resource whose base (wave-uniform, in scalar registers) moves one
// k-step at a time and whose size ends at the chunk's last column: a column
// past kc, or a row past nrows (its offset is pushed out of range), reads
// as zero, with no branch and no per-load address arithmetic in the vector
// unit.  The compiler then counts the loads in flight exactly, so each
// k-step waits only for its own load, PF loads behind the newest.
template <class T, int PFN = 8>
struct ARing {
  static constexpr int PF = PFN;
  typename MM<T>::C v[PF];
  const char* base;   // row row0 of the next load's first column (wave-uniform)
  int step;           // bytes per k-step: 4 columns
  int left;           // bytes of the chunk from base on (<= 0: none left)
  unsigned voff;      // the lane's offset: row i of column kk, or out of range
  int kc;
};

// Hardware word 3 of a raw buffer resource on this architecture family.
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ const char* uniform_ptr(const void* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<const char*>(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ void buf_load(float2& out, __amdgpu_buffer_rsrc_t r, unsigned voff) {
  typedef float v2f __attribute__((ext_vector_type(2)));
  const v2f v = __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
  out = make_float2(v.x, v.y);
}
__device__ __forceinline__ void buf_load(double2& out, __amdgpu_buffer_rsrc_t r, unsigned voff) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  const v2d v = __builtin_bit_cast(v2d, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
  out = make_double2(v.x, v.y);
}

template <class T, int PF>
__device__ __forceinline__ void ring_load(ARing<T, PF>& g, int u) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(g.base), 0, max(g.left, 0), kBufWord3);
  buf_load(g.v[u], r, g.voff);
  g.base += g.step;
  g.left -= g.step;
}

template <class T, int PF>
__device__ __forceinline__ void mm_prime(ARing<T, PF>& g, const typename MM<T>::C* __restrict__ A,
                                         long long lda, int row0, int nrows, int k_lo, int kc) {
  using C = typename MM<T>::C;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kk = lane >> 4;
  row0 = __builtin_amdgcn_readfirstlane(row0);
  g.base = uniform_ptr(A + row0 + (long long)k_lo * lda);
  g.step = (int)(4 * lda * (long long)sizeof(C));
  g.left = (int)(((long long)kc * lda - row0) * (long long)sizeof(C));
  g.voff = row0 + i < nrows ? (unsigned)((i + kk * lda) * (long long)sizeof(C)) : 0x80000000u;
  g.kc = kc;
#pragma unroll
  for (int u = 0; u < PF; ++u) ring_load(g, u);
}

// The FP32 accumulators flush into the FP64 sums every FL k-steps (kFlush
// unless the caller chooses another), whatever the depth of the ring, so
// that every ring gives the same sums.
constexpr int kFlush = 8;

template <class T, int NT, int PF, int FL = kFlush>
__device__ __forceinline__ void mm_run(Acc<T, NT>& acc, ARing<T, PF>& g,
                                       const typename MM<T>::C* __restrict__ Bs, int bst) {
  static_assert(PF % FL == 0 || FL % PF == 0, "ring depth and flush interval");
  const int kk = (threadIdx.x & 63) >> 4;
  const int kc = g.kc;
  const int nsteps = (kc + 3) >> 2;
  const typename MM<T>::C* Bk = Bs + kk * bst;
  const int bstep = 4 * bst;
  int s0 = 0;
  for (; s0 + PF <= nsteps; s0 += PF) {
    if (FL > PF && s0 > 0 && s0 % FL == 0) acc.flush();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const typename MM<T>::C a = g.v[u];
      ring_load(g, u);
      mma_step<T, NT>(acc, a, Bk);
      Bk += bstep;
      if (FL <= PF && u % FL == FL - 1) acc.flush();
    }
  }
  if (FL > PF && s0 > 0 && s0 % FL == 0 && s0 < nsteps) acc.flush();
#pragma unroll
  for (int u = 0; u < PF; ++u)
    if (s0 + u < nsteps) {
      mma_step<T, NT>(acc, g.v[u], Bk);
      Bk += bstep;
      if (FL <= PF && u % FL == FL - 1) acc.flush();
    }
  acc.flush();
}

// One wave: acc += A[its 16-row tile, columns k_lo .. k_lo+kc) * Bs[0..kc).
// A points at row 0 of the operator (column-major, leading dimension lda >=
// nrows); rows >= nrows and columns >= kc read as 0.  Bs holds kc rows
// rounded up to a multiple of 4, zero-padded, with row stride bst.
//
// A complex tile product is four real MFMAs into two accumulators:
//   re += a.re b.re,  im += a.re b.im,  re += (-a.im) b.im,  im += a.im b.re,
// ordered so that the two MFMAs feeding one accumulator are not adjacent.
// Each k-step of 4 columns needs one complex A entry per lane from HBM; a
// ring of PF registers keeps the next PF k-steps' loads in flight while
// the current MFMAs run, so a wave does not stall on HBM latency.
template <class T, int NT, int PF = 8, int FL = kFlush>
__device__ __forceinline__ void mm_chunk(Acc<T, NT>& acc, const typename MM<T>::C* __restrict__ A,
                                         long long lda, int row0, int nrows, int k_lo, int kc,
                                         const typename MM<T>::C* __restrict__ Bs, int bst) {
  ARing<T, PF> g;
  mm_prime(g, A, lda, row0, nrows, k_lo, kc);
  mm_run<T, NT, PF, FL>(acc, g, Bs, bst);
}

// The dispatcher hands blocks to the eight XCDs in turn (block b to XCD
// b mod 8), and each XCD has an L2 of its own.  Blocks that share an operand
// (the row groups of one product share its B, the RHS tiles share its A) sit
// at consecutive logical indices; this renumbering gives every XCD one
// contiguous run of logical indices, taken in order, so that such blocks
// meet in one L2 instead of each fetching the operand from HBM.  A bijection
// of [0, gridDim.x) for any grid size.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, n = gridDim.x;
  const int x = b & 7, s = b >> 3, q = n >> 3, rm = n & 7;
  return x < rm ? x * (q + 1) + s : rm * (q + 1) + (x - rm) * q + s;
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
        c.x = T(acc.vre(t, v));
        c.y = T(acc.vim(t, v));
        f(row, t * 16 + (lane & 15), c);
      }
    }
}

constexpr int kKC = 64;  // k-chunk of B staged in LDS

// k-chunk of the four-wave merge blocks: 128 columns of FP32 B (17 or 34 KiB
// of LDS), so that a wave's operator ring drains at a chunk end half as
// often; 64 of FP64 (the static LDS limit); one-wave blocks take 32.
template <class T, int WV>
constexpr int merge_kc() { return WV == 4 ? (sizeof(T) == 4 ? 2 * kKC : kKC) : 32; }

// ---- leaf upward: g from the sources, w = W g, h = N_i w -------------------------
// block = (leaf, rhs tile, group of pole_group poles); it stages the source
// fields of its element and right-hand sides once in LDS, then walks its
// poles: g_m = k1 X1 + k2 X2 + k3 X3 (or the residual gin), w = W_m g on the
// matrix cores, h = N_i w from an LDS copy of w (w_lds) or from memory.
// XL: the source fields are staged in LDS once per block (else read per pole).
template <class T, int NT, bool XL>
__device__ __forceinline__ void leaf_up_body(const MmLeafUpArgs<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1, LRT = NT == 2 ? 5 : 4;   // LRT = log2(RT)
  extern __shared__ unsigned char smem[];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const int G = a.pole_group, npg = (a.npole + G - 1) / G;
  int rest = bid;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pg = rest % npg;
  const int leaf = rest / npg;
  const int p_lo = pg * G, p_hi = min(a.npole, p_lo + G);
  const int q = a.q, q2 = q * q, q2p = (q2 + 3) & ~3;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs, ns = a.nsrc;
  C* gs = reinterpret_cast<C*>(smem);                        // g [q2p][BST]
  C* wl = gs + q2p * BST;                                    // w tile [q2][RT]
  T* xs = reinterpret_cast<T*>(wl + (a.w_lds ? q2 * RT : 0));   // sources [ns][q2p][RT] (x_lds)
  const bool xl = XL && !a.gin;
  T* nrl = xs + (xl ? ns * q2p * RT : 0);                    // normal-derivative rows [2q]
  int* hmt = reinterpret_cast<int*>(nrl + 2 * q);            // edge slot -> side | t << 2
  if (xl) {
    // k fastest so that the state reads are contiguous (one-time divisions)
    for (int idx = threadIdx.x; idx < ns * RT * q2p; idx += blockDim.x) {
      const int k = idx % q2p, fj = idx / q2p;
      const int j = fj % RT, f = fj / RT;
      const int rhs = rt * RT + j;
      T v = T(0);
      if (k < q2 && rhs < r)
        v = T(a.state[rhs * a.rhs_stride + (long long)f * a.n_int + (long long)L.elem * q2 + k]);
      xs[(f * q2p + k) * RT + j] = v;
    }
  }
  for (int t = threadIdx.x; t < 2 * q; t += blockDim.x) nrl[t] = T(a.nrow[t]);
  for (int k = threadIdx.x; k < L.e; k += blockDim.x) {
    const int slot = k / q;
    int sd = -1, seen = -1;
    for (int m = 0; m < 4; ++m)
      if ((L.side_mask >> m) & 1)
        if (++seen == slot) { sd = m; break; }
    hmt[k] = sd | ((k - slot * q) << 2);
  }
  const int wave = threadIdx.x >> 6;
  for (int pole = p_lo; pole < p_hi; ++pole) {
    // g of this pole, rhs fastest (all LDS, or contiguous gin rows)
    if (a.gin) {
      const C* gp = a.gin + ((long long)pole * a.w_pole + (long long)leaf * q2) * r + rt * RT;
      for (int idx = threadIdx.x; idx < q2p * RT; idx += blockDim.x) {
        const int j = idx & (RT - 1), k = idx >> LRT;
        C g;
        g.x = g.y = T(0);
        if (k < q2 && rt * RT + j < r) g = gp[(long long)k * r + j];
        gs[k * BST + j] = g;
      }
    } else if (!XL) {
      // sources read from memory (k fastest: contiguous state rows)
      __syncthreads();
      const PoleCoef pc = a.coef[pole];
      for (int idx = threadIdx.x; idx < q2p * RT; idx += blockDim.x) {
        const int j = idx / q2p, k = idx - j * q2p;
        const int rhs = rt * RT + j;
        C g;
        g.x = g.y = T(0);
        if (k < q2 && rhs < r) {
          // sources rounded to T as when staged, so that both ways give
          // the same g (the FP64 residual of the precision form corrects it)
          const double* x1 = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
          const double u1 = double(T(x1[k])), u2 = double(T(x1[a.n_int + k]));
          const double u3 = ns > 2 ? double(T(x1[2 * a.n_int + k])) : 0.0;
          g.x = T(fma(pc.k1.x, u1, fma(pc.k2.x, u2, pc.k3.x * u3)));
          g.y = T(fma(pc.k1.y, u1, fma(pc.k2.y, u2, pc.k3.y * u3)));
        }
        gs[k * BST + j] = g;
      }
    } else {
      __syncthreads();   // sources staged / previous pole done with gs
      const PoleCoef pc = a.coef[pole];
      for (int idx = threadIdx.x; idx < q2p * RT; idx += blockDim.x) {
        const int j = idx & (RT - 1), k = idx >> LRT;
        const double u1 = double(xs[k * RT + j]), u2 = double(xs[(q2p + k) * RT + j]);
        const double u3 = ns > 2 ? double(xs[(2 * q2p + k) * RT + j]) : 0.0;
        C g;
        g.x = T(fma(pc.k1.x, u1, fma(pc.k2.x, u2, pc.k3.x * u3)));
        g.y = T(fma(pc.k1.y, u1, fma(pc.k2.y, u2, pc.k3.y * u3)));
        gs[k * BST + j] = g;
      }
    }
    __syncthreads();
    const C* W = a.ops + pole * a.pole_stride + L.op_off;
    C* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
    for (int tile = wave; tile * 16 < q2; tile += kBlock / 64) {
      Acc<T, NT> acc;
      acc.zero();
      // (products of depth q^2 <= 256: FP64 flushes every 16 k-steps suffice)
      mm_chunk<T, NT, 8, 16>(acc, W, q2, tile * 16, q2, 0, q2, gs, BST);
      mm_emit<T, NT>(acc, tile * 16, q2, [&](int row, int j, C c) {
        const int rhs = rt * RT + j;
        if (rhs < r) w[(long long)row * r + rhs] = c;
        if (a.w_lds) wl[row * RT + j] = c;
      });
    }
    __syncthreads();
    C* h = a.h + ((long long)pole * a.h_pole + L.vec_off) * r;
    for (int idx = threadIdx.x; idx < L.e * RT; idx += blockDim.x) {
      const int j = idx & (RT - 1), re = idx >> LRT;
      const int rhs = rt * RT + j;
      if (rhs >= r) continue;
      const int hm = hmt[re], sd = hm & 3, t = hm >> 2;
      const T* nr = nrl + ((sd == 1 || sd == 3) ? q : 0);
      const T sc = T((sd == 0) ? -a.sx : (sd == 1) ? a.sx : (sd == 2) ? -a.sy : a.sy);
      T sx_ = T(0), sy_ = T(0);
      for (int k = 0; k < q; ++k) {
        const int node = (sd < 2) ? (k + q * t) : (t + q * k);
        const C wv = a.w_lds ? wl[node * RT + j] : w[(long long)node * r + rhs];
        sx_ += nr[k] * wv.x;
        sy_ += nr[k] * wv.y;
      }
      C hv;
      hv.x = sc * sx_;
      hv.y = sc * sy_;
      h[(long long)re * r + rhs] = hv;
    }
    if (a.gin) __syncthreads();   // the next pole's gin staging overwrites gs
  }
}

template <class T, int NT, bool XL>
__global__ __launch_bounds__(kBlock) void k_leaf_up_mm(MmLeafUpArgs<T> a) {
  leaf_up_body<T, NT, XL>(a, xcd_block());
}

template <class T, int NT, bool XL>
__global__ __launch_bounds__(kBlock) void k_leaf_up_mm_multi(Multi<MmLeafUpArgs<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmLeafUpArgs<T> a = m.args[i];
  leaf_up_body<T, NT, XL>(a, bid);
}

// ---- merge upward: g3 = h3a + h3b (- j3), h_par = [h1a; h2b] - Y g3 ----------
// block = (box, group of poles, rhs tile, row group of 16 x WV rows of Y)
template <class T, int NT, int WV>
__device__ __forceinline__ void merge_up_body(const MmMergeArgs<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  constexpr int RB = 16 * WV, KC = merge_kc<T, WV>();  // rows per block, k-chunk
  __shared__ C Bs[KC * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  const int G = a.pole_group, npg = (a.npole + G - 1) / G;
  int rest = bid;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pg = rest % npg;
  const int box = rest / npg;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2;
  if (rg > 0 && rg * RB >= ext) return;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const int* ja = a.idx + B.j_off;
  const int r = a.nrhs;
  const int row0 = rg * RB + (threadIdx.x >> 6) * 16;
  const int lane = threadIdx.x & 63;
  // child vector positions of this lane's output rows (h1 of child a, h2 of
  // child b), the same for every pole
  int bo[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = row0 + MM<T>::row(lane, v);
    bo[v] = row >= ext ? 0 : row < n1 ? B.a_vec + i1[row] : B.b_vec + i2[row - n1];
  }
  // the interface rows' child positions (and flux slots), the same for every
  // pole, held in LDS so that the staging's gathers wait on one LDS read
  constexpr int kIdxLds = 256;
  __shared__ int sidx[4 * kIdxLds];
  const bool sl = n3 <= kIdxLds;
  if (sl) {
    for (int t = threadIdx.x; t < n3; t += blockDim.x) {
      sidx[t] = i3a[t];
      sidx[kIdxLds + t] = i3b[t];
      if (a.dn) {
        sidx[2 * kIdxLds + t] = ja[t];
        sidx[3 * kIdxLds + t] = ja[n3 + t];
      }
    }
    __syncthreads();
  }
  const int p_end = min(a.npole, (pg + 1) * G);
  for (int pole = pg * G; pole < p_end; ++pole) {
    const C* hc = a.child + (long long)pole * a.child_pole * r;
    C* g3 = a.g3 + ((long long)pole * a.g3_pole + B.g3_off) * r;
    const C* Y = a.ops + pole * a.pole_stride + B.op_off + (long long)n3 * (ext + n3);
    // the epilogue's base values, loaded first so that their latency
    // overlaps the staging and the products
    C basev[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        basev[t][v].x = basev[t][v].y = T(0);
        const int row = row0 + MM<T>::row(lane, v);
        const int rhs = rt * RT + t * 16 + (lane & 15);
        if (row < ext && rhs < r) basev[t][v] = hc[(long long)bo[v] * r + rhs];
      }
    Acc<T, NT> acc;
    acc.zero();
    // each chunk's operator loads are issued before its B is staged
    ARing<T> ring;
    if (row0 < ext) mm_prime(ring, Y, ext, row0, ext, 0, min(KC, n3));
    for (int k0 = 0; k0 < n3; k0 += KC) {
      const int kc = min(KC, n3 - k0), kcp = (kc + 3) & ~3;
      for (int idx = threadIdx.x; idx < kcp * RT; idx += blockDim.x) {
        const int k = idx / RT, j = idx - k * RT;
        const int rhs = rt * RT + j;
        C v;
        v.x = v.y = T(0);
        if (k < kc && rhs < r) {
          const int kg = k0 + k;
          const int ia = sl ? sidx[kg] : i3a[kg], ib = sl ? sidx[kIdxLds + kg] : i3b[kg];
          const C x = hc[(long long)(B.a_vec + ia) * r + rhs];
          const C y = hc[(long long)(B.b_vec + ib) * r + rhs];
          v.x = x.x + y.x;
          v.y = x.y + y.y;
          if (a.dn) {
            // flux rows of the correction: du/dn(a) + du/dn(b) = -(dn_a + dn_b),
            // which enters as g3 = h3a + h3b + dn_a + dn_b
            const double2* dp = a.dn + (long long)pole * a.dn_pole * r;
            const int sa = sl ? sidx[2 * kIdxLds + kg] : ja[kg];
            const int sb = sl ? sidx[3 * kIdxLds + kg] : ja[n3 + kg];
            const double2 da = dp[(long long)sa * r + rhs];
            const double2 db = dp[(long long)sb * r + rhs];
            v.x += T(da.x + db.x);
            v.y += T(da.y + db.y);
          }
          if (rg == 0) g3[(long long)(k0 + k) * r + rhs] = v;
        }
        Bs[k * BST + j] = v;
      }
      __syncthreads();
      if (row0 < ext) mm_run<T, NT>(acc, ring, Bs, BST);
      __syncthreads();
      if (row0 < ext && k0 + KC < n3) mm_prime(ring, Y, ext, row0, ext, k0 + KC, min(KC, n3 - k0 - KC));
    }
    if (row0 < ext) {
      C* hp = a.self + ((long long)pole * a.self_pole + B.vec_off) * r;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + MM<T>::row(lane, v);
          const int rhs = rt * RT + t * 16 + (lane & 15);
          if (row < ext && rhs < r) {
            C o;
            o.x = T(double(basev[t][v].x) - acc.vre(t, v));
            o.y = T(double(basev[t][v].y) - acc.vim(t, v));
            hp[(long long)row * r + rhs] = o;
          }
        }
    }
  }
}

template <class T, int NT, int WV = 4>
__global__ __launch_bounds__(64 * WV) void k_merge_up_mm(MmMergeArgs<T> a) {
  merge_up_body<T, NT, WV>(a, xcd_block());
}

template <class T, int NT, int WV = 4>
__global__ __launch_bounds__(64 * WV) void k_merge_up_mm_multi(Multi<MmMergeArgs<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmMergeArgs<T> a = m.args[i];
  merge_up_body<T, NT, WV>(a, bid);
}

// ---- merge downward: u3 = -Z [u_ext; g3], scattered to the children --------
template <class T, int NT, int WV>
__device__ __forceinline__ void merge_down_body(const MmMergeArgs<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  constexpr int RB = 16 * WV, KC = merge_kc<T, WV>();  // rows per block, k-chunk
  __shared__ C Bs[KC * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = bid;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int box = rest / a.npole;
  const BoxDesc B = a.boxes[box];
  const int n1 = B.n1, n2 = B.n2, n3 = B.n3, ext = n1 + n2, m = ext + n3;
  if (rg * RB >= n3) return;
  const int* i1 = a.idx + B.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + n2;
  const int* i3b = i3a + n3;
  const int r = a.nrhs;
  const C* up = a.self + ((long long)pole * a.self_pole + B.vec_off) * r;
  const C* g3 = a.g3 + ((long long)pole * a.g3_pole + B.g3_off) * r;
  C* uc = a.child + (long long)pole * a.child_pole * r;
  const int row0 = rg * RB + (threadIdx.x >> 6) * 16;
  const int lane = threadIdx.x & 63;
  // child positions of this lane's output rows, fetched before the staging
  int ia[4], ib[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = row0 + MM<T>::row(lane, v);
    ia[v] = row < n3 ? i3a[row] : 0;
    ib[v] = row < n3 ? i3b[row] : 0;
  }
  // each chunk's operator loads are issued before its B is staged; row group
  // 0 also copies the exterior values it stages to the children (one read
  // of u_ext serves both: a separate copy pass re-read it from HBM)
  const C* Z = a.ops + pole * a.pole_stride + B.op_off;
  ARing<T> ring;
  if (row0 < n3) mm_prime(ring, Z, n3, row0, n3, 0, min(KC, m));
  Acc<T, NT> acc;
  acc.zero();
  for (int k0 = 0; k0 < m; k0 += KC) {
    const int kc = min(KC, m - k0), kcp = (kc + 3) & ~3;
    for (int idx = threadIdx.x; idx < kcp * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = rt * RT + j;
      C v;
      v.x = v.y = T(0);
      if (k < kc && rhs < r) {
        const int kg = k0 + k;
        if (kg < ext) {
          v = up[(long long)kg * r + rhs];
          if (rg == 0)
            uc[(long long)(kg < n1 ? B.a_vec + i1[kg] : B.b_vec + i2[kg - n1]) * r + rhs] = v;
        } else {
          v = g3[(long long)(kg - ext) * r + rhs];
        }
      }
      Bs[k * BST + j] = v;
    }
    __syncthreads();
    if (row0 < n3) mm_run<T, NT>(acc, ring, Bs, BST);
    __syncthreads();
    if (row0 < n3 && k0 + KC < m) mm_prime(ring, Z, n3, row0, n3, k0 + KC, min(KC, m - k0 - KC));
  }
  if (row0 >= n3) return;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + MM<T>::row(lane, v);
      const int rhs = rt * RT + t * 16 + (lane & 15);
      if (row < n3 && rhs < r) {
        C u3;
        u3.x = T(-acc.vre(t, v));
        u3.y = T(-acc.vim(t, v));
        uc[(long long)(B.a_vec + ia[v]) * r + rhs] = u3;
        uc[(long long)(B.b_vec + ib[v]) * r + rhs] = u3;
      }
    }
}

template <class T, int NT, int WV = 4>
__global__ __launch_bounds__(64 * WV) void k_merge_down_mm(MmMergeArgs<T> a) {
  merge_down_body<T, NT, WV>(a, xcd_block());
}

template <class T, int NT, int WV = 4>
__global__ __launch_bounds__(64 * WV) void k_merge_down_mm_multi(Multi<MmMergeArgs<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmMergeArgs<T> a = m.args[i];
  merge_down_body<T, NT, WV>(a, bid);
}

// ---- two merge levels per launch ----------------------------------------------
// A block takes one level-(l+1) box T, one pole and one RHS tile.  Upward,
// the four level-(l-1) vectors under T are read once into LDS, the two
// level-l merges write their h into LDS, and T's merge reads it from
// there: only the g3 of both levels and T's h go to HBM.  Downward, T's u3
// and exterior values go straight into the staged operands of its two
// children, whose merges write the level-(l-1) vectors.  Every product,
// staging and rounding is the one the per-level kernels perform, so the
// results are bit-identical to two per-level launches.

// Fields of one of two boxes, chosen by a wave-uniform index (no dynamic
// indexing of a register array).
struct BoxPair {
  BoxDesc d0, d1;
  __device__ const BoxDesc& operator[](int b) const { return b ? d1 : d0; }
};

template <class T, int NT>
__device__ __forceinline__ void merge2_up_body(const MmMerge2Args<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  extern __shared__ unsigned char smem[];
  C* const lds = reinterpret_cast<C*>(smem);
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = bid;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int top = rest / a.npole;
  const BoxDesc Tb = a.hi[top];
  BoxPair P;
  P.d0 = a.lo[Tb.a_box];
  P.d1 = a.lo[Tb.b_box];
  const int r = a.nrhs, c0 = rt * RT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  // LDS: the four child vectors X [rows][RT], the two level-l outputs Y
  // [rows][RT], the staged g3 operands S [rows][BST]
  const int ce0 = P.d0.n1 + P.d0.n3, ce1 = P.d0.n2 + P.d0.n3;
  const int ce2 = P.d1.n1 + P.d1.n3, ce3 = P.d1.n2 + P.d1.n3;
  const int xo1 = ce0, xo2 = xo1 + ce1, xo3 = xo2 + ce2, nx = xo3 + ce3;
  const int eA = P.d0.n1 + P.d0.n2, eB = P.d1.n1 + P.d1.n2;
  C* const X = lds;
  C* const Y = X + nx * RT;
  C* const S = Y + (eA + eB) * RT;
  const int pA = (P.d0.n3 + 3) & ~3;
  const int tA = (eA + 15) >> 4, tB = (eB + 15) >> 4;
  const int n1 = Tb.n1, n3 = Tb.n3, ext = Tb.n1 + Tb.n2;
  const C* YT = a.ops + pole * a.pole_stride + Tb.op_off + (long long)n3 * (ext + n3);
  // the operator loads of this wave's first tile of each level are issued
  // first, so that they are in flight while the vectors are loaded
  ARing<T> ring0, ringT;
  if (wave < tA + tB) {
    const int b = wave < tA ? 0 : 1;
    const BoxDesc& D = P[b];
    const int e = D.n1 + D.n2;
    mm_prime(ring0, a.ops + pole * a.pole_stride + D.op_off + (long long)D.n3 * (e + D.n3), e,
             (wave - (b ? tA : 0)) * 16, e, 0, D.n3);
  }
  if (wave * 16 < ext) mm_prime(ringT, YT, ext, wave * 16, ext, 0, n3);
  const C* hc = a.child + (long long)pole * a.child_pole * r;
  for (int idx = threadIdx.x; idx < nx * RT; idx += blockDim.x) {
    const int k = idx / RT, j = idx - k * RT;
    const int vec = k < xo1 ? P.d0.a_vec + k
                  : k < xo2 ? P.d0.b_vec + (k - xo1)
                  : k < xo3 ? P.d1.a_vec + (k - xo2) : P.d1.b_vec + (k - xo3);
    C v;
    v.x = v.y = T(0);
    if (c0 + j < r) v = hc[(long long)vec * r + c0 + j];
    X[idx] = v;
  }
  __syncthreads();
  const double2* dp = a.dn ? a.dn + (long long)pole * a.dn_pole * r : nullptr;
  // g3 of the two level-l boxes: h3a + h3b (+ the flux residual)
  for (int b = 0; b < 2; ++b) {
    const BoxDesc& D = P[b];
    const int* i3a = a.idx + D.idx_off + D.n1 + D.n2;
    const int* i3b = i3a + D.n3;
    const int* ja = a.idx + D.j_off;
    const C* xa = X + (b ? xo2 : 0) * RT;
    const C* xb = X + (b ? xo3 : xo1) * RT;
    C* Sb = S + (b ? pA * BST : 0);
    C* g3 = a.g3_lo + ((long long)pole * a.g3_lo_pole + D.g3_off) * r;
    const int pb = (D.n3 + 3) & ~3;
    for (int idx = threadIdx.x; idx < pb * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = c0 + j;
      C v;
      v.x = v.y = T(0);
      if (k < D.n3 && rhs < r) {
        const C x = xa[i3a[k] * RT + j];
        const C y = xb[i3b[k] * RT + j];
        v.x = x.x + y.x;
        v.y = x.y + y.y;
        if (dp) {
          const double2 da = dp[(long long)ja[k] * r + rhs];
          const double2 db = dp[(long long)ja[D.n3 + k] * r + rhs];
          v.x += T(da.x + db.x);
          v.y += T(da.y + db.y);
        }
        g3[(long long)k * r + rhs] = v;
      }
      Sb[k * BST + j] = v;
    }
  }
  __syncthreads();
  // the level-l products, 16-row tiles of both boxes over the waves
  {
    for (int tile = wave; tile < tA + tB; tile += nw) {
      const int b = tile < tA ? 0 : 1;
      const BoxDesc& D = P[b];
      const int ext = D.n1 + D.n2, row0 = (tile - (b ? tA : 0)) * 16;
      const C* Yop = a.ops + pole * a.pole_stride + D.op_off + (long long)D.n3 * (ext + D.n3);
      Acc<T, NT> acc;
      acc.zero();
      if (tile != wave) mm_prime(ring0, Yop, ext, row0, ext, 0, D.n3);
      mm_run<T, NT>(acc, ring0, S + (b ? pA * BST : 0), BST);
      const int* i1 = a.idx + D.idx_off;
      const int* i2 = i1 + D.n1;
      const C* xa = X + (b ? xo2 : 0) * RT;
      const C* xb = X + (b ? xo3 : xo1) * RT;
      C* yo = Y + (b ? eA : 0) * RT;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + MM<T>::row(lane, v);
          const int j = t * 16 + (lane & 15);
          if (row < ext) {
            const C base = row < D.n1 ? xa[i1[row] * RT + j] : xb[i2[row - D.n1] * RT + j];
            C o;
            o.x = T(double(base.x) - acc.vre(t, v));
            o.y = T(double(base.y) - acc.vim(t, v));
            yo[row * RT + j] = o;
          }
        }
    }
  }
  __syncthreads();
  // T: g3 from the level-l outputs, then its product into HBM
  const int* i1 = a.idx + Tb.idx_off;
  const int* i2 = i1 + n1;
  const int* i3a = i2 + Tb.n2;
  const int* i3b = i3a + n3;
  {
    const int* ja = a.idx + Tb.j_off;
    C* g3 = a.g3_hi + ((long long)pole * a.g3_hi_pole + Tb.g3_off) * r;
    const int pt = (n3 + 3) & ~3;
    for (int idx = threadIdx.x; idx < pt * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = c0 + j;
      C v;
      v.x = v.y = T(0);
      if (k < n3 && rhs < r) {
        const C x = Y[i3a[k] * RT + j];
        const C y = Y[(eA + i3b[k]) * RT + j];
        v.x = x.x + y.x;
        v.y = x.y + y.y;
        if (dp) {
          const double2 da = dp[(long long)ja[k] * r + rhs];
          const double2 db = dp[(long long)ja[n3 + k] * r + rhs];
          v.x += T(da.x + db.x);
          v.y += T(da.y + db.y);
        }
        g3[(long long)k * r + rhs] = v;
      }
      S[k * BST + j] = v;
    }
  }
  __syncthreads();
  C* hp = a.self + ((long long)pole * a.self_pole + Tb.vec_off) * r;
  for (int tile = wave; tile * 16 < ext; tile += nw) {
    const int row0 = tile * 16;
    Acc<T, NT> acc;
    acc.zero();
    if (tile != wave) mm_prime(ringT, YT, ext, row0, ext, 0, n3);
    mm_run<T, NT>(acc, ringT, S, BST);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + MM<T>::row(lane, v);
        const int j = t * 16 + (lane & 15);
        if (row < ext && c0 + j < r) {
          const C base = row < n1 ? Y[i1[row] * RT + j] : Y[(eA + i2[row - n1]) * RT + j];
          C o;
          o.x = T(double(base.x) - acc.vre(t, v));
          o.y = T(double(base.y) - acc.vim(t, v));
          hp[(long long)row * r + c0 + j] = o;
        }
      }
  }
}

template <class T, int NT>
__device__ __forceinline__ void merge2_down_body(const MmMerge2Args<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  extern __shared__ unsigned char smem[];
  C* const lds = reinterpret_cast<C*>(smem);
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = bid;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int top = rest / a.npole;
  const BoxDesc Tb = a.hi[top];
  BoxPair P;
  P.d0 = a.lo[Tb.a_box];
  P.d1 = a.lo[Tb.b_box];
  const int r = a.nrhs, c0 = rt * RT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  // LDS: T's operand [u_ext; g3] and the children's [u_ext; g3], [rows][BST]
  const int extT = Tb.n1 + Tb.n2, mT = extT + Tb.n3, mpT = (mT + 3) & ~3;
  const int eA = P.d0.n1 + P.d0.n2, mA = eA + P.d0.n3, mpA = (mA + 3) & ~3;
  const int eB = P.d1.n1 + P.d1.n2, mB = eB + P.d1.n3, mpB = (mB + 3) & ~3;
  C* const PT = lds;
  C* const SA = PT + mpT * BST;
  C* const SB = SA + mpA * BST;
  const int tA = (P.d0.n3 + 15) >> 4, tB = (P.d1.n3 + 15) >> 4;
  const C* ZT = a.ops + pole * a.pole_stride + Tb.op_off;
  // the operator loads of this wave's first tile of each level are issued
  // first, so that they are in flight while the operands are loaded
  ARing<T> ringT, ring0;
  if (wave * 16 < Tb.n3) mm_prime(ringT, ZT, Tb.n3, wave * 16, Tb.n3, 0, mT);
  if (wave < tA + tB) {
    const int b = wave < tA ? 0 : 1;
    const BoxDesc& D = P[b];
    mm_prime(ring0, a.ops + pole * a.pole_stride + D.op_off, D.n3, (wave - (b ? tA : 0)) * 16, D.n3, 0,
             b ? mB : mA);
  }
  {
    const C* up = a.self + ((long long)pole * a.self_pole + Tb.vec_off) * r;
    const C* g3 = a.g3_hi + ((long long)pole * a.g3_hi_pole + Tb.g3_off) * r;
    for (int idx = threadIdx.x; idx < mpT * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = c0 + j;
      C v;
      v.x = v.y = T(0);
      if (k < mT && rhs < r) v = k < extT ? up[(long long)k * r + rhs] : g3[(long long)(k - extT) * r + rhs];
      PT[k * BST + j] = v;
    }
  }
  for (int b = 0; b < 2; ++b) {
    const BoxDesc& D = P[b];
    const int e = b ? eB : eA, m = b ? mB : mA, mp = b ? mpB : mpA;
    C* Sb = b ? SB : SA;
    const C* g3 = a.g3_lo + ((long long)pole * a.g3_lo_pole + D.g3_off) * r;
    for (int idx = threadIdx.x; idx < (mp - e) * RT; idx += blockDim.x) {
      const int k = e + idx / RT, j = idx % RT;
      const int rhs = c0 + j;
      C v;
      v.x = v.y = T(0);
      if (k < m && rhs < r) v = g3[(long long)(k - e) * r + rhs];
      Sb[k * BST + j] = v;
    }
  }
  __syncthreads();
  const int* i1 = a.idx + Tb.idx_off;
  const int* i2 = i1 + Tb.n1;
  const int* i3a = i2 + Tb.n2;
  const int* i3b = i3a + Tb.n3;
  // T's exterior values to the children's exterior rows
  for (int idx = threadIdx.x; idx < extT * RT; idx += blockDim.x) {
    const int k = idx / RT, j = idx - k * RT;
    const C v = PT[k * BST + j];
    if (k < Tb.n1) SA[i1[k] * BST + j] = v;
    else SB[i2[k - Tb.n1] * BST + j] = v;
  }
  // T's u3 = -Z [u_ext; g3] to the children's interface rows
  {
    for (int tile = wave; tile * 16 < Tb.n3; tile += nw) {
      const int row0 = tile * 16;
      Acc<T, NT> acc;
      acc.zero();
      if (tile != wave) mm_prime(ringT, ZT, Tb.n3, row0, Tb.n3, 0, mT);
      mm_run<T, NT>(acc, ringT, PT, BST);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + MM<T>::row(lane, v);
          const int j = t * 16 + (lane & 15);
          if (row < Tb.n3) {
            C u3;
            u3.x = T(-acc.vre(t, v));
            u3.y = T(-acc.vim(t, v));
            SA[i3a[row] * BST + j] = u3;
            SB[i3b[row] * BST + j] = u3;
          }
        }
    }
  }
  __syncthreads();
  // the level-l boxes: exterior values and u3 into the level l-1 vectors
  C* uc = a.child + (long long)pole * a.child_pole * r;
  for (int b = 0; b < 2; ++b) {
    const BoxDesc& D = P[b];
    const int e = b ? eB : eA;
    const C* Sb = b ? SB : SA;
    const int* j1 = a.idx + D.idx_off;
    const int* j2 = j1 + D.n1;
    for (int idx = threadIdx.x; idx < e * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = c0 + j;
      if (rhs >= r) continue;
      const C v = Sb[k * BST + j];
      if (k < D.n1) uc[(long long)(D.a_vec + j1[k]) * r + rhs] = v;
      else uc[(long long)(D.b_vec + j2[k - D.n1]) * r + rhs] = v;
    }
  }
  {
    for (int tile = wave; tile < tA + tB; tile += nw) {
      const int b = tile < tA ? 0 : 1;
      const BoxDesc& D = P[b];
      const int row0 = (tile - (b ? tA : 0)) * 16;
      const int m = b ? mB : mA;
      const C* Z = a.ops + pole * a.pole_stride + D.op_off;
      Acc<T, NT> acc;
      acc.zero();
      if (tile != wave) mm_prime(ring0, Z, D.n3, row0, D.n3, 0, m);
      mm_run<T, NT>(acc, ring0, b ? SB : SA, BST);
      const int* j3a = a.idx + D.idx_off + D.n1 + D.n2;
      const int* j3b = j3a + D.n3;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + MM<T>::row(lane, v);
          const int rhs = c0 + t * 16 + (lane & 15);
          if (row < D.n3 && rhs < r) {
            C u3;
            u3.x = T(-acc.vre(t, v));
            u3.y = T(-acc.vim(t, v));
            uc[(long long)(D.a_vec + j3a[row]) * r + rhs] = u3;
            uc[(long long)(D.b_vec + j3b[row]) * r + rhs] = u3;
          }
        }
    }
  }
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_merge2_up_mm(MmMerge2Args<T> a) {
  merge2_up_body<T, NT>(a, xcd_block());
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_merge2_up_mm_multi(Multi<MmMerge2Args<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmMerge2Args<T> a = m.args[i];
  merge2_up_body<T, NT>(a, bid);
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_merge2_down_mm(MmMerge2Args<T> a) {
  merge2_down_body<T, NT>(a, xcd_block());
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_merge2_down_mm_multi(Multi<MmMerge2Args<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmMerge2Args<T> a = m.args[i];
  merge2_down_body<T, NT>(a, bid);
}

template <class T>
size_t merge2_up_lds_bytes(int nt, int child_rows, int mid_rows, int stage_rows) {
  const int RT = 16 * nt;
  return sizeof(typename MM<T>::C) *
         ((size_t)RT * (child_rows + mid_rows) + (size_t)(RT + 1) * stage_rows);
}

template <class T>
size_t merge2_down_lds_bytes(int nt, int rows) {
  return sizeof(typename MM<T>::C) * (size_t)(16 * nt + 1) * rows;
}

// ---- leaf downward: y = w - S u_e (in place of w) -----------------------------
template <class T, int NT>
__device__ __forceinline__ void leaf_down_body(const MmLeafDownArgs<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[4 * (kMaxP - 2) * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = bid;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt; rest /= n_rt;
  const int pole = rest % a.npole;
  const int leaf = rest / a.npole;
  const int q2 = a.q * a.q;
  if (rg * 64 >= q2) return;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs, e = L.e, ep = (e + 3) & ~3;
  const C* ue = a.u + ((long long)pole * a.u_pole + L.vec_off) * r;
  const int row0 = rg * 64 + (threadIdx.x >> 6) * 16;
  const int lane = threadIdx.x & 63;
  const C* S = a.ops + pole * a.pole_stride + L.op_off + (long long)q2 * q2;
  C* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
  C* yo = a.y0 ? a.y0 + ((long long)pole * a.w_pole + (long long)leaf * q2) * r : w;
  // this lane's w entries and the operator loads are issued before the
  // staging, so that the block waits for memory once
  C wv[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + MM<T>::row(lane, v);
      const int rhs = rt * RT + t * 16 + (lane & 15);
      wv[t][v].x = wv[t][v].y = T(0);
      if (row < q2 && rhs < r) wv[t][v] = w[(long long)row * r + rhs];
    }
  ARing<T> ring;
  if (row0 < q2 && e > 0) mm_prime(ring, S, q2, row0, q2, 0, e);
  for (int idx = threadIdx.x; idx < ep * RT; idx += blockDim.x) {
    const int k = idx / RT, j = idx - k * RT;
    const int rhs = rt * RT + j;
    C v;
    v.x = v.y = T(0);
    if (k < e && rhs < r) v = ue[(long long)k * r + rhs];
    Bs[k * BST + j] = v;
  }
  __syncthreads();
  if (row0 >= q2) return;
  Acc<T, NT> acc;
  acc.zero();
  if (e > 0) mm_run<T, NT>(acc, ring, Bs, BST);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + MM<T>::row(lane, v);
      const int rhs = rt * RT + t * 16 + (lane & 15);
      if (row < q2 && rhs < r) {
        C o = wv[t][v];
        o.x -= T(acc.vre(t, v));
        o.y -= T(acc.vim(t, v));
        yo[(long long)row * r + rhs] = o;
      }
    }
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_down_mm(MmLeafDownArgs<T> a) {
  leaf_down_body<T, NT>(a, xcd_block());
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_down_mm_multi(Multi<MmLeafDownArgs<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmLeafDownArgs<T> a = m.args[i];
  leaf_down_body<T, NT>(a, bid);
}

// ---- leaf downward fused with the pole sum ----------------------------------------
// block = (leaf, rhs tile, row group); it walks the poles in order:
//   y_m = w_m - S_m u_e,m,  u' = sum_m Re(cu_m y_m),  v' = (beta u0 + sum_m Re(cv_m y_m)) / tau,
// so the per-pole solutions never go back to HBM.  Accumulation is FP64.
template <class T, int NT>
__device__ __forceinline__ void leaf_down_sum_body(const MmLeafDownArgs<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[4 * (kMaxP - 2) * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = bid;
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
    const C* S = a.ops + pole * a.pole_stride + L.op_off + (long long)q2 * q2;
    const C* w = a.w + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
    const C* y0 = a.y0 ? a.y0 + ((long long)pole * a.w_pole + (long long)leaf * q2) * r : nullptr;
    // this pole's w (and first-sweep y) entries of the lane and its operator
    // loads are issued before the staging: one wait for memory per pole
    C wv[NT][4], y0v[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + MM<T>::row(lane, v);
        const int rhs = rt * RT + t * 16 + (lane & 15);
        wv[t][v].x = wv[t][v].y = T(0);
        y0v[t][v].x = y0v[t][v].y = T(0);
        if (row < q2 && rhs < r) {
          wv[t][v] = w[(long long)row * r + rhs];
          // corrected solution of the precision form: y0 + (w - S u_e)
          if (y0) y0v[t][v] = y0[(long long)row * r + rhs];
        }
      }
    ARing<T> ring;
    if (row0 < q2 && e > 0) mm_prime(ring, S, q2, row0, q2, 0, e);
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
      Acc<T, NT> acc;
      acc.zero();
      if (e > 0) mm_run<T, NT>(acc, ring, Bs, BST);
      const PoleCoef pc = a.coef[pole];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + MM<T>::row(lane, v);
          const int rhs = rt * RT + t * 16 + (lane & 15);
          if (row < q2 && rhs < r) {
            double yr = double(wv[t][v].x) - acc.vre(t, v);
            double yi = double(wv[t][v].y) - acc.vim(t, v);
            if (y0) {
              yr += double(y0v[t][v].x);
              yi += double(y0v[t][v].y);
            }
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

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_down_sum_mm(MmLeafDownArgs<T> a) {
  leaf_down_sum_body<T, NT>(a, xcd_block());
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_leaf_down_sum_mm_multi(Multi<MmLeafDownArgs<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const MmLeafDownArgs<T> a = m.args[i];
  leaf_down_sum_body<T, NT>(a, bid);
}

// ---- shallow water: wall values at the root ------------------------------------
//   eta_b = Q (rhs_b - a h_root),  rhs_b = (a n.v0 - f t.v0) / (c tau)
// block = (pole, rhs tile, row group of 64 wall slots)
template <class T, int NT>
__device__ __forceinline__ void sw_root_body(const SwRootArgs<T>& a, const int bid) {
  using C = typename MM<T>::C;
  constexpr int RT = 16 * NT, BST = RT + 1;
  __shared__ C Bs[kKC * BST];
  const int n_rt = (a.nrhs + RT - 1) / RT;
  int rest = bid;
  const int rg = rest % a.row_groups; rest /= a.row_groups;
  const int rt = rest % n_rt;
  const int pole = rest / n_rt;
  const int n = a.n, r = a.nrhs;
  const double2 al = a.coef[pole].alpha;
  const double ax = al.x * a.inv_tau, ay = al.y * a.inv_tau;   // a = alpha / tau
  const double sc = a.inv_tau * a.inv_c;
  const C* h = a.h + (long long)pole * n * r;
  const C* Q = a.ops + pole * a.pole_stride + a.q_off;
  const int row0 = rg * 64 + (threadIdx.x >> 6) * 16;
  Acc<T, NT> acc;
  acc.zero();
  for (int k0 = 0; k0 < n; k0 += kKC) {
    const int kc = min(kKC, n - k0), kcp = (kc + 3) & ~3;
    for (int idx = threadIdx.x; idx < kcp * RT; idx += blockDim.x) {
      const int k = idx / RT, j = idx - k * RT;
      const int rhs = rt * RT + j;
      C v;
      v.x = v.y = T(0);
      if (k < kc && rhs < r) {
        const C hv = h[(long long)(k0 + k) * r + rhs];
        double br, bi;   // wall-row right-hand side
        if (a.rw) {
          const double2 w = a.rw[((long long)pole * a.rw_pole + a.wall_info[k0 + k].w) * r + rhs];
          br = w.x;
          bi = w.y;
        } else {
          const double nv = a.wall[(long long)rhs * 2 * n + k0 + k];
          const double tv = a.wall[(long long)rhs * 2 * n + n + k0 + k];
          br = (ax * nv - a.f * tv) * sc;
          bi = ay * nv * sc;
        }
        v.x = T(br - (ax * double(hv.x) - ay * double(hv.y)));
        v.y = T(bi - (ax * double(hv.y) + ay * double(hv.x)));
      }
      Bs[k * BST + j] = v;
    }
    __syncthreads();
    if (row0 < n) mm_chunk<T, NT>(acc, Q, n, row0, n, k0, kc, Bs, BST);
    __syncthreads();
  }
  if (row0 >= n) return;
  C* u = a.u + (long long)pole * n * r;
  mm_emit<T, NT>(acc, row0, n, [&](int row, int j, C c) {
    const int rhs = rt * RT + j;
    if (rhs < r) u[(long long)row * r + rhs] = c;
  });
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_sw_root_mm(SwRootArgs<T> a) {
  sw_root_body<T, NT>(a, xcd_block());
}

template <class T, int NT>
__global__ __launch_bounds__(kBlock) void k_sw_root_mm_multi(Multi<SwRootArgs<T>> m) {
  int i;
  const int bid = m.locate(xcd_block(), i);
  const SwRootArgs<T> a = m.args[i];
  sw_root_body<T, NT>(a, bid);
}



// ---- launchers -----------------------------------------------------------------

template <class T, int NT>
size_t leaf_up_lds(int q, bool with_w = false, int nsrc_staged = 0) {
  const size_t q2 = (size_t)q * q, q2p = (q2 + 3) & ~(size_t)3, RT = 16 * NT;
  return sizeof(typename MM<T>::C) * (q2p * (RT + 1) + (with_w ? q2 * RT : 0)) +
         sizeof(T) * ((size_t)nsrc_staged * q2p * RT + 2 * (size_t)q) + sizeof(int) * 4 * (size_t)q;
}

// ---- multi-instance launchers ------------------------------------------------------

template <class T>
size_t leaf_up_lds_bytes(int q, int nt, bool with_w, int nsrc_staged) {
  return nt == 2 ? leaf_up_lds<T, 2>(q, with_w, nsrc_staged) : leaf_up_lds<T, 1>(q, with_w, nsrc_staged);
}

template <class K>
static hipError_t allow_lds(K* kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <class T, int NT, bool XL>
static hipError_t leaf_up_launch(const MmLeafUpArgs<T>* a, const Multi<MmLeafUpArgs<T>>* m,
                                 int blocks, size_t lds, hipStream_t s) {
  if (a) {
    const hipError_t e = allow_lds(&k_leaf_up_mm<T, NT, XL>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_leaf_up_mm<T, NT, XL>), dim3(blocks), dim3(kBlock), lds, s, *a);
  } else {
    const hipError_t e = allow_lds(&k_leaf_up_mm_multi<T, NT, XL>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_leaf_up_mm_multi<T, NT, XL>), dim3(blocks), dim3(kBlock), lds, s, *m);
  }
  return hipGetLastError();
}

template <class T>
static hipError_t leaf_up_dispatch(const MmLeafUpArgs<T>* a, const Multi<MmLeafUpArgs<T>>* m,
                                   int blocks, int nt, bool xl, size_t lds, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (nt == 2) return xl ? leaf_up_launch<T, 2, true>(a, m, blocks, lds, s)
                         : leaf_up_launch<T, 2, false>(a, m, blocks, lds, s);
  return xl ? leaf_up_launch<T, 1, true>(a, m, blocks, lds, s)
            : leaf_up_launch<T, 1, false>(a, m, blocks, lds, s);
}

template <class T>
hipError_t launch_leaf_up_mm_multi(const Multi<MmLeafUpArgs<T>>& m, int blocks, int nt, bool xl,
                                   size_t lds, hipStream_t s) {
  return leaf_up_dispatch<T>(nullptr, &m, blocks, nt, xl, lds, s);
}

#define HX_MULTI_LAUNCHER(NAME, ARGS)                                                          \
  template <class T>                                                                           \
  hipError_t launch_##NAME##_multi(const Multi<ARGS<T>>& m, int blocks, int nt, hipStream_t s) { \
    if (blocks <= 0) return hipSuccess;                                                        \
    if (nt == 2) hipLaunchKernelGGL((k_##NAME##_multi<T, 2>), dim3(blocks), dim3(kBlock), 0, s, m); \
    else hipLaunchKernelGGL((k_##NAME##_multi<T, 1>), dim3(blocks), dim3(kBlock), 0, s, m);   \
    return hipGetLastError();                                                                  \
  }
HX_MULTI_LAUNCHER(leaf_down_mm, MmLeafDownArgs)
HX_MULTI_LAUNCHER(leaf_down_sum_mm, MmLeafDownArgs)
HX_MULTI_LAUNCHER(sw_root_mm, SwRootArgs)
#undef HX_MULTI_LAUNCHER

// Single-instance launches with the arguments by value (a group of one
// instance skips the table lookup), same block counts as the multi form.
template <class T>
hipError_t launch_leaf_up_mm_one(const MmLeafUpArgs<T>& a, int blocks, int nt, size_t lds, hipStream_t s) {
  return leaf_up_dispatch<T>(&a, nullptr, blocks, nt, a.x_lds != 0, lds, s);
}

#define HX_ONE_LAUNCHER(NAME, ARGS)                                                            \
  template <class T>                                                                           \
  hipError_t launch_##NAME##_one(const ARGS<T>& a, int blocks, int nt, hipStream_t s) {        \
    if (blocks <= 0) return hipSuccess;                                                        \
    if (nt == 2) hipLaunchKernelGGL((k_##NAME<T, 2>), dim3(blocks), dim3(kBlock), 0, s, a);    \
    else hipLaunchKernelGGL((k_##NAME<T, 1>), dim3(blocks), dim3(kBlock), 0, s, a);           \
    return hipGetLastError();                                                                  \
  }
HX_ONE_LAUNCHER(leaf_down_mm, MmLeafDownArgs)
HX_ONE_LAUNCHER(leaf_down_sum_mm, MmLeafDownArgs)
HX_ONE_LAUNCHER(sw_root_mm, SwRootArgs)
#undef HX_ONE_LAUNCHER

// Merge launches: wv waves per block (4: 64 rows per block, 1: 16 rows).
#define HX_MERGE_LAUNCHERS(NAME)                                                                   \
  template <class T>                                                                               \
  hipError_t launch_##NAME##_multi(const Multi<MmMergeArgs<T>>& m, int blocks, int nt, int wv,     \
                                   hipStream_t s) {                                                \
    if (blocks <= 0) return hipSuccess;                                                            \
    if (wv == 1) {                                                                                 \
      if (nt == 2) hipLaunchKernelGGL((k_##NAME##_multi<T, 2, 1>), dim3(blocks), dim3(64), 0, s, m); \
      else hipLaunchKernelGGL((k_##NAME##_multi<T, 1, 1>), dim3(blocks), dim3(64), 0, s, m);       \
    } else {                                                                                       \
      if (nt == 2) hipLaunchKernelGGL((k_##NAME##_multi<T, 2, 4>), dim3(blocks), dim3(kBlock), 0, s, m); \
      else hipLaunchKernelGGL((k_##NAME##_multi<T, 1, 4>), dim3(blocks), dim3(kBlock), 0, s, m);   \
    }                                                                                              \
    return hipGetLastError();                                                                      \
  }                                                                                                \
  template <class T>                                                                               \
  hipError_t launch_##NAME##_one(const MmMergeArgs<T>& a, int blocks, int nt, int wv, hipStream_t s) { \
    if (blocks <= 0) return hipSuccess;                                                            \
    if (wv == 1) {                                                                                 \
      if (nt == 2) hipLaunchKernelGGL((k_##NAME<T, 2, 1>), dim3(blocks), dim3(64), 0, s, a);       \
      else hipLaunchKernelGGL((k_##NAME<T, 1, 1>), dim3(blocks), dim3(64), 0, s, a);               \
    } else {                                                                                       \
      if (nt == 2) hipLaunchKernelGGL((k_##NAME<T, 2, 4>), dim3(blocks), dim3(kBlock), 0, s, a);   \
      else hipLaunchKernelGGL((k_##NAME<T, 1, 4>), dim3(blocks), dim3(kBlock), 0, s, a);           \
    }                                                                                              \
    return hipGetLastError();                                                                      \
  }
HX_MERGE_LAUNCHERS(merge_up_mm)
HX_MERGE_LAUNCHERS(merge_down_mm)
#undef HX_MERGE_LAUNCHERS

#define HX_MERGE2_LAUNCHERS(NAME)                                                                  \
  template <class T>                                                                               \
  hipError_t launch_##NAME##_multi(const Multi<MmMerge2Args<T>>& m, int blocks, int nt, size_t lds, \
                                   hipStream_t s) {                                                \
    if (blocks <= 0) return hipSuccess;                                                            \
    if (nt == 2) hipLaunchKernelGGL((k_##NAME##_multi<T, 2>), dim3(blocks), dim3(kBlock), lds, s, m); \
    else hipLaunchKernelGGL((k_##NAME##_multi<T, 1>), dim3(blocks), dim3(kBlock), lds, s, m);      \
    return hipGetLastError();                                                                      \
  }                                                                                                \
  template <class T>                                                                               \
  hipError_t launch_##NAME##_one(const MmMerge2Args<T>& a, int blocks, int nt, size_t lds,         \
                                 hipStream_t s) {                                                  \
    if (blocks <= 0) return hipSuccess;                                                            \
    if (nt == 2) hipLaunchKernelGGL((k_##NAME<T, 2>), dim3(blocks), dim3(kBlock), lds, s, a);      \
    else hipLaunchKernelGGL((k_##NAME<T, 1>), dim3(blocks), dim3(kBlock), lds, s, a);              \
    return hipGetLastError();                                                                      \
  }
HX_MERGE2_LAUNCHERS(merge2_up_mm)
HX_MERGE2_LAUNCHERS(merge2_down_mm)
#undef HX_MERGE2_LAUNCHERS

#define HX_INST(T)                                                                                     \
  template size_t leaf_up_lds_bytes<T>(int, int, bool, int);                                                      \
  template hipError_t launch_leaf_up_mm_multi<T>(const Multi<MmLeafUpArgs<T>>&, int, int, bool, size_t, hipStream_t); \
  template hipError_t launch_merge_up_mm_multi<T>(const Multi<MmMergeArgs<T>>&, int, int, int, hipStream_t);   \
  template hipError_t launch_merge_down_mm_multi<T>(const Multi<MmMergeArgs<T>>&, int, int, int, hipStream_t); \
  template hipError_t launch_leaf_down_mm_multi<T>(const Multi<MmLeafDownArgs<T>>&, int, int, hipStream_t); \
  template hipError_t launch_leaf_down_sum_mm_multi<T>(const Multi<MmLeafDownArgs<T>>&, int, int, hipStream_t); \
  template hipError_t launch_sw_root_mm_multi<T>(const Multi<SwRootArgs<T>>&, int, int, hipStream_t);   \
  template hipError_t launch_leaf_up_mm_one<T>(const MmLeafUpArgs<T>&, int, int, size_t, hipStream_t);    \
  template hipError_t launch_merge_up_mm_one<T>(const MmMergeArgs<T>&, int, int, int, hipStream_t);            \
  template hipError_t launch_merge_down_mm_one<T>(const MmMergeArgs<T>&, int, int, int, hipStream_t);          \
  template hipError_t launch_leaf_down_mm_one<T>(const MmLeafDownArgs<T>&, int, int, hipStream_t);        \
  template hipError_t launch_leaf_down_sum_mm_one<T>(const MmLeafDownArgs<T>&, int, int, hipStream_t);    \
  template hipError_t launch_sw_root_mm_one<T>(const SwRootArgs<T>&, int, int, hipStream_t);          \
  template hipError_t launch_merge2_up_mm_multi<T>(const Multi<MmMerge2Args<T>>&, int, int, size_t, hipStream_t); \
  template hipError_t launch_merge2_down_mm_multi<T>(const Multi<MmMerge2Args<T>>&, int, int, size_t, hipStream_t); \
  template hipError_t launch_merge2_up_mm_one<T>(const MmMerge2Args<T>&, int, int, size_t, hipStream_t);   \
  template hipError_t launch_merge2_down_mm_one<T>(const MmMerge2Args<T>&, int, int, size_t, hipStream_t); \
  template size_t merge2_up_lds_bytes<T>(int, int, int, int);                                       \
  template size_t merge2_down_lds_bytes<T>(int, int);
HX_INST(float)
HX_INST(double)
#undef HX_INST


}  // namespace hx
