// Shallow water with slip walls: the parts of the step that differ from the
// wave equation.  The solver itself (element, merge and root operators) is
// the same hierarchical solve of a shifted Laplacian, with the wall nodes
// kept as exterior unknowns up to the root.
//
// Per step, for every right-hand side (state v1, v2, eta on interior nodes):
//   k_sw_prep   eta, div(v) and curl(v) = d_x v2 - d_y v1 on the interior
//               nodes, by differentiation along interior lines through the
//               q = p-2 interior values (the source of every pole's
//               right-hand side);
//   k_sw_wall   n.v and t.v at every wall node, the interior line normal to
//               the wall extrapolated to the wall node;
// per pole (leaf and merge sweeps as for the wave, then the root):
//   root        eta_b = Q (rhs_b - a h_root), Q = (a T_root - f D_t)^{-1};
// after the sweeps:
//   k_sw_post   the pole sums E0 = sum b eta, E1 = sum b (a/s) eta,
//               E2 = sum b eta/s on each element's full grid (interior from
//               the leaf sweep, edges from the merge sweep; in the precision
//               form added to the first sweep's sums), then
//               eta' = E0,
//               v' = c grad(E1) - c f J grad(E2) - (beta1 v0 - f beta2 J v0)/tau,
//               with beta1 = sum b a/s, beta2 = sum b/s (all m); grad uses the
//               element's p-point lines.
#include "hx_kernels.h"

namespace hx {

__device__ __forceinline__ void sw_prep_body(const SwPrepArgs& a, const int bid) {
  __shared__ double Dq[(kMaxP - 2) * (kMaxP - 2)];
  const int leaf = bid / a.nrhs;
  const int rhs = bid - leaf * a.nrhs;
  const int q = a.q, q2 = q * q;
  for (int t = threadIdx.x; t < q2; t += blockDim.x) Dq[t] = a.Dq[t];
  __syncthreads();
  const long long e0 = (long long)leaf * q2;
  const double* v1 = a.state + rhs * a.rhs_stride + e0;
  const double* v2 = v1 + a.n_int;
  const double* eta = v2 + a.n_int;
  double* out = a.prep + rhs * a.rhs_stride + e0;   // fields eta, div, curl
  for (int k = threadIdx.x; k < q2; k += blockDim.x) {
    const int i = k % q, j = k / q;
    double d1x = 0, d1y = 0, d2x = 0, d2y = 0;
    for (int m = 0; m < q; ++m) {
      d1x += Dq[i * q + m] * v1[m + q * j];
      d2x += Dq[i * q + m] * v2[m + q * j];
      d1y += Dq[j * q + m] * v1[i + q * m];
      d2y += Dq[j * q + m] * v2[i + q * m];
    }
    out[k] = eta[k];
    out[a.n_int + k] = a.sx * d1x + a.sy * d2y;
    out[2 * a.n_int + k] = a.sx * d2x - a.sy * d1y;
  }
}

__global__ __launch_bounds__(kBlock) void k_sw_prep(SwPrepArgs a) { sw_prep_body(a, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void k_sw_prep_multi(Multi<SwPrepArgs> m) {
  int i;
  const int bid = m.locate(blockIdx.x, i);
  const SwPrepArgs a = m.args[i];
  sw_prep_body(a, bid);
}

__device__ __forceinline__ void sw_wall_body(const SwWallArgs& a, const int bid) {
  const long long idx = (long long)bid * blockDim.x + threadIdx.x;
  if (idx >= (long long)a.n_wall * a.nrhs) return;
  const int rhs = (int)(idx / a.n_wall);
  const int k = (int)(idx - (long long)rhs * a.n_wall);
  const int4 wi = a.wall[k];                       // element, side, node along the side
  const int q = a.q, q2 = q * q;
  const double* v1 = a.state + rhs * a.rhs_stride + (long long)wi.x * q2;
  const double* v2 = v1 + a.n_int;
  const int side = wi.y, t = wi.z;
  const double* w = (side == 0 || side == 2) ? a.w_lo : a.w_hi;
  double e1 = 0, e2 = 0;
  for (int m = 0; m < q; ++m) {
    const int node = (side < 2) ? (m + q * t) : (t + q * m);
    e1 += w[m] * v1[node];
    e2 += w[m] * v2[node];
  }
  // n and t = (-n2, n1): left (-1,0),(0,-1); right (1,0),(0,1);
  // bottom (0,-1),(1,0); top (0,1),(-1,0).  Written as sign arithmetic: an
  // if/else chain here was compiled with the top wall's t.v sign lost.
  const double sg = (side == 0 || side == 2) ? -1.0 : 1.0;   // outward sign
  const bool xs = side < 2;                                 // normal along x
  const double nv = sg * (xs ? e1 : e2);
  const double tv = xs ? sg * e2 : -sg * e1;
  a.out[(long long)rhs * 2 * a.n_wall + k] = nv;
  a.out[(long long)rhs * 2 * a.n_wall + a.n_wall + k] = tv;
}

__global__ __launch_bounds__(kBlock) void k_sw_wall(SwWallArgs a) { sw_wall_body(a, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void k_sw_wall_multi(Multi<SwWallArgs> m) {
  int i;
  const int bid = m.locate(blockIdx.x, i);
  const SwWallArgs a = m.args[i];
  sw_wall_body(a, bid);
}

// G = a T_root - f D_t for every pole of a build chunk (column-major n x n).
__global__ __launch_bounds__(kBlock) void k_sw_root_form(SwRootFormArgs a) {
  const int j = blockIdx.y;
  const long long nn = (long long)a.n * a.n;
  const double2* T = a.T + j * a.T_stride;
  double2* G = a.G + j * nn;
  const double2 al = a.a[j];
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nn;
       f += (long long)gridDim.x * blockDim.x) {
    const double2 t = T[f];
    G[f] = make_double2(al.x * t.x - al.y * t.y - a.f * a.Dt[f], al.x * t.y + al.y * t.x);
  }
}

// Side (0 left, 1 right, 2 bottom, 3 top) -> position among the element's
// edge slots, -1 when the side carries no exterior values.
__device__ __forceinline__ int sw_slot_of_side(int mask, int side) {
  return ((mask >> side) & 1) ? __popc(mask & ((1 << side) - 1)) : -1;
}

// block = (element, group of RR right-hand sides).  Phase 1: every thread
// owns up to kPer (node, rhs) items of the element's full grid, rhs fastest
// so that the pole values of RR consecutive right-hand sides are read
// together, and sums them over the poles in registers (the next pole's
// values are fetched before the current ones are added).  Phase 2: the
// sums go to LDS, and every interior item forms the gradients along the
// p-point lines and the new state.
template <class T>
__device__ __forceinline__ void sw_post_body(const SwPostArgs<T>& a, const int bid) {
  const int RR = a.RR;
  using C = typename Cplx<T>::type;
  constexpr int kPer = 8;
  extern __shared__ double smem[];
  const int p = a.p, q = a.q, q2 = q * q, pp = p * p;
  const int nrg = (a.nrhs + RR - 1) / RR;
  const int rg = bid % nrg;
  const int leaf = bid / nrg;
  const int r = a.nrhs, r0 = rg * RR, ES = RR + 1;
  const LeafDesc L = a.leaves[leaf];
  double* Ds = smem;                  // p x p
  double* E = Ds + pp;                // [3][p*p][ES]: E0, E1, E2
  for (int t = threadIdx.x; t < pp; t += blockDim.x) Ds[t] = a.D[t];
  const C* yb = a.y + (long long)leaf * q2 * r + r0;
  const C* ub = a.ue + (long long)L.vec_off * r + r0;
  int off[kPer];                      // >= 0: interior (y) offset; < -1: edge (ue) offset -2-off
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    off[u] = -1;
    if (idx < RR * pp) {
      const int node = idx / RR, jr = idx - node * RR;
      const int i = node % p, j = node / p;
      if (r0 + jr < r) {
        const bool ix = (i > 0 && i < p - 1), iy = (j > 0 && j < p - 1);
        if (ix && iy) {
          off[u] = ((i - 1) + q * (j - 1)) * r + jr;
        } else if (ix != iy) {
          const int sd = (i == 0) ? 0 : (i == p - 1) ? 1 : (j == 0) ? 2 : 3;
          const int t = (sd < 2) ? j - 1 : i - 1;
          const int sl = sw_slot_of_side(L.side_mask, sd);
          if (sl >= 0) off[u] = -2 - ((sl * q + t) * r + jr);
        }
      }
    }
  }
  auto fetch = [&](int pole, C* buf) {
    const C* yp = yb + (long long)pole * a.y_pole * r;
    const C* up = ub + (long long)pole * a.e_pole * r;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      C v;
      v.x = v.y = T(0);
      if (off[u] >= 0) v = yp[off[u]];
      else if (off[u] < -1) v = up[-2 - off[u]];
      buf[u] = v;
    }
  };
  double e0[kPer], e1[kPer], e2[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) e0[u] = e1[u] = e2[u] = 0.0;
  C cur[kPer], nxt[kPer];
  fetch(0, nxt);
  for (int pole = 0; pole < a.npole; ++pole) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) cur[u] = nxt[u];
    if (pole + 1 < a.npole) fetch(pole + 1, nxt);
    const SwCoef c = a.coef[pole];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const double yr = double(cur[u].x), yi = double(cur[u].y);
      e0[u] += c.c0.x * yr - c.c0.y * yi;
      e1[u] += c.c1.x * yr - c.c1.y * yi;
      e2[u] += c.c2.x * yr - c.c2.y * yi;
    }
  }
  // precision form: add the first sweep's sums [leaf][3][p*p][rhs]
  const double* es = a.esum ? a.esum + (long long)leaf * 3 * pp * r + r0 : nullptr;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    if (idx < RR * pp) {
      const int node = idx / RR, jr = idx - node * RR;
      double f0 = e0[u], f1 = e1[u], f2 = e2[u];
      if (es && r0 + jr < r) {
        f0 += es[(long long)node * r + jr];
        f1 += es[(long long)(pp + node) * r + jr];
        f2 += es[(long long)(2 * pp + node) * r + jr];
      }
      E[node * ES + jr] = f0;
      E[(pp + node) * ES + jr] = f1;
      E[(2 * pp + node) * ES + jr] = f2;
    }
  }
  __syncthreads();
  // interior items, node fastest (the state is [rhs][field][n_int])
  const double c = a.c, f = a.f;
  for (int idx = threadIdx.x; idx < RR * q2; idx += blockDim.x) {
    const int jr = idx / q2, k = idx - jr * q2;
    if (r0 + jr >= r) break;
    const int i = k % q + 1, j = k / q + 1;
    double e1x = 0, e1y = 0, e2x = 0, e2y = 0;
    for (int m = 0; m < p; ++m) {
      const double dx = Ds[i * p + m], dy = Ds[j * p + m];
      e1x += dx * E[(pp + m + p * j) * ES + jr];
      e2x += dx * E[(2 * pp + m + p * j) * ES + jr];
      e1y += dy * E[(pp + i + p * m) * ES + jr];
      e2y += dy * E[(2 * pp + i + p * m) * ES + jr];
    }
    e1x *= a.sx; e2x *= a.sx; e1y *= a.sy; e2y *= a.sy;
    double* st = a.state + (long long)(r0 + jr) * a.rhs_stride + (long long)L.elem * q2;
    const double v1 = st[k], v2 = st[a.n_int + k];
    st[k] = c * e1x - c * f * e2y - (a.beta1 * v1 - f * a.beta2 * v2) * a.inv_tau;
    st[a.n_int + k] = c * e1y + c * f * e2x - (a.beta1 * v2 + f * a.beta2 * v1) * a.inv_tau;
    st[2 * a.n_int + k] = E[(i + p * j) * ES + jr];
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_sw_post(SwPostArgs<T> a) { sw_post_body<T>(a, blockIdx.x); }

template <class T>
__global__ __launch_bounds__(kBlock) void k_sw_post_multi(Multi<SwPostArgs<T>> m) {
  int i;
  const int bid = m.locate(blockIdx.x, i);
  const SwPostArgs<T> a = m.args[i];
  sw_post_body<T>(a, bid);
}



hipError_t launch_sw_root_form(const SwRootFormArgs& a, int chunk, hipStream_t s) {
  const long long nn = (long long)a.n * a.n;
  long long bx = (nn + kBlock - 1) / kBlock;
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_sw_root_form, dim3((unsigned)bx, chunk), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Right-hand sides per block: a power of two up to 8, the grid items of one
// pole at most 8 per thread.
int sw_post_rr(int p, int nrhs) {
  int RR = 8;
  while (RR > 1 && (RR / 2 >= nrhs || RR * p * p > 8 * kBlock)) RR /= 2;
  return RR;
}

size_t sw_post_lds_bytes(int p, int RR) { return sizeof(double) * (size_t)p * p * (1 + 3 * (RR + 1)); }


template <class T>
hipError_t launch_sw_post_multi(const Multi<SwPostArgs<T>>& m, int blocks, size_t lds, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sw_post_multi<T>), dim3(blocks), dim3(kBlock), lds, s, m);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sw_post_one(const SwPostArgs<T>& a, int blocks, size_t lds, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sw_post<T>), dim3(blocks), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}
template hipError_t launch_sw_post_one<double>(const SwPostArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_sw_post_one<float>(const SwPostArgs<float>&, int, size_t, hipStream_t);

hipError_t launch_sw_prep_one(const SwPrepArgs& a, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sw_prep, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sw_wall_one(const SwWallArgs& a, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sw_wall, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sw_prep_multi(const Multi<SwPrepArgs>& m, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sw_prep_multi, dim3(blocks), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_sw_wall_multi(const Multi<SwWallArgs>& m, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sw_wall_multi, dim3(blocks), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}

template hipError_t launch_sw_post_multi<double>(const Multi<SwPostArgs<double>>&, int, size_t, hipStream_t);
template hipError_t launch_sw_post_multi<float>(const Multi<SwPostArgs<float>>&, int, size_t, hipStream_t);


}  // namespace hx
