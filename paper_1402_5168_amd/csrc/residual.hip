// FP64 residual of the collocation equations (precision form).
//
// After the FP32 sweep every pole has a solution y0 on the element interiors
// and values u_e on the element edges.  Assembled on an element's full
// p x p grid (zero on a Dirichlet boundary), they give, in FP64,
//   * the residual of the PDE rows at the interior nodes (section 2.2):
//       res = g - (sx^2 Dx C^2 Dx + sy^2 Dy C^2 Dy - sigma) y,
//     g = k1 X1 + k2 X2 (+ k3 X3) from the source fields X of the step;
//   * the element's outward normal derivative at each of its edge slots;
//     the flux rows' residual at an interface node is minus the sum of its
//     two elements' values, added by the merge of the correction sweep;
//   * shallow water: at a wall slot, the residual of the oblique wall row,
//       rhs_b - (a d_n y - f d_t y),  rhs_b = (a n.v0 - f t.v0)/(tau c),
//     stored in place of the normal derivative (a wall node has one element),
//     and the first sweep's pole sums E0, E1, E2 on the element's full grid,
//     kept in registers across the poles and written once.
// One block per (element, group of RR right-hand sides) walks the poles;
// the sources, the grid values and the row operators live in LDS.
#include "hx_kernels.h"

namespace hx {

// Position of side s among the element's interface sides, -1 if it lies on
// the outer boundary.
__device__ __forceinline__ int slot_of_side(int mask, int s) {
  return ((mask >> s) & 1) ? __popc(mask & ((1 << s) - 1)) : -1;
}

// Side (0 left, 1 right, 2 bottom, 3 top) holding the given slot.
__device__ __forceinline__ int side_of_slot_r(int mask, int slot) {
  int seen = -1;
  for (int k = 0; k < 4; ++k)
    if ((mask >> k) & 1)
      if (++seen == slot) return k;
  return -1;
}

template <bool SW>
__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs a, int RR) {
  extern __shared__ double sm[];
  const int p = a.p, q = a.q, q2 = q * q, pp = p * p;
  const int nrg = (a.nrhs + RR - 1) / RR;
  const int rg = blockIdx.x % nrg;
  const int leaf = blockIdx.x / nrg;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs;
  const int r0 = rg * RR;                             // first right-hand side of the group
  double* Ds = sm;
  double* cs = Ds + pp;
  // row operators of the element: Mx[jj][i][l] = sx^2 sum_m D[i][m] c2(m,jj) D[m][l]
  // (interior row jj, interior i, all l) and My[i][jj][l] likewise along columns
  double* Mx = cs + pp;
  double* My = Mx + q2 * p;
  const int ns = a.nsrc;
  double* st = My + q2 * p;                           // sources: [nsrc][q*q][RR]
  double2* U = reinterpret_cast<double2*>(st + ns * RR * q2);   // grid values [p*p][RR]
  for (int t = threadIdx.x; t < pp; t += blockDim.x) {
    Ds[t] = a.D[t];
    cs[t] = a.c2[(long long)L.elem * pp + t];
  }
  for (int idx = threadIdx.x; idx < RR * ns * q2; idx += blockDim.x) {
    const int k = idx / RR, jr = idx - k * RR;        // k < nsrc q^2: field-major
    const int fld = k / q2, kk = k - fld * q2;
    const int rhs = r0 + jr;
    st[idx] = (rhs < r) ? a.state[rhs * a.rhs_stride + (long long)fld * a.n_int +
                                  (long long)L.elem * q2 + kk]
                        : 0.0;
  }
  __syncthreads();
  const double sx2 = a.sx * a.sx, sy2 = a.sy * a.sy;
  for (int idx = threadIdx.x; idx < q2 * p; idx += blockDim.x) {
    const int l = idx % p, ij = idx / p;               // ij = (row) * q + (col), interior
    const int i = ij % q + 1, jj = ij / q + 1;
    double mx = 0.0, my = 0.0;
    for (int m = 0; m < p; ++m) {
      mx += Ds[i * p + m] * cs[m + p * jj] * Ds[m * p + l];
      my += Ds[jj * p + m] * cs[i + p * m] * Ds[m * p + l];
    }
    Mx[((jj - 1) * q + (i - 1)) * p + l] = sx2 * mx;
    My[((i - 1) * q + (jj - 1)) * p + l] = sy2 * my;
  }
  const double itau = 1.0 / a.tau;
  // grid values of one pole, fetched a pole ahead into registers (at most
  // kPer per thread) so their HBM latency overlaps the previous pole's work
  constexpr int kPer = 8;
  auto fetch = [&](int pole, float2* buf) {
    const float2* y0 = a.y0 + ((long long)pole * a.w_pole + (long long)leaf * q2) * r + r0;
    const float2* ue = a.ue + ((long long)pole * a.e_pole + L.vec_off) * r + r0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = threadIdx.x + u * kBlock;
      float2 v = make_float2(0.f, 0.f);
      if (idx < RR * pp) {
        const int node = idx / RR, jr = idx - node * RR;
        const int i = node % p, jj = node / p;
        if (r0 + jr < r) {
          const bool ix = (i > 0 && i < p - 1), iy = (jj > 0 && jj < p - 1);
          if (ix && iy) {
            v = y0[(long long)((i - 1) + q * (jj - 1)) * r + jr];
          } else if (ix != iy) {  // non-corner edge node
            const int s = (i == 0) ? 0 : (i == p - 1) ? 1 : (jj == 0) ? 2 : 3;
            const int t = (s < 2) ? jj - 1 : i - 1;
            const int sl = slot_of_side(L.side_mask, s);
            if (sl >= 0) v = ue[(long long)(sl * q + t) * r + jr];
          }
        }
      }
      buf[u] = v;
    }
  };
  float2 nxt[kPer];
  double e0[SW ? kPer : 1], e1[SW ? kPer : 1], e2[SW ? kPer : 1];   // pole sums, SW only
  if constexpr (SW) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) e0[u] = e1[u] = e2[u] = 0.0;
  }
  fetch(0, nxt);
  for (int pole = 0; pole < a.npole; ++pole) {
    __syncthreads();   // row operators ready / previous pole done with U
    SwCoef sc3;
    if constexpr (SW) sc3 = a.swc[pole];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = threadIdx.x + u * kBlock;
      if (idx < RR * pp) {
        U[idx] = make_double2(nxt[u].x, nxt[u].y);
        if constexpr (SW) {
          const double yr = nxt[u].x, yi = nxt[u].y;
          e0[u] += sc3.c0.x * yr - sc3.c0.y * yi;
          e1[u] += sc3.c1.x * yr - sc3.c1.y * yi;
          e2[u] += sc3.c2.x * yr - sc3.c2.y * yi;
        }
      }
    }
    __syncthreads();
    if (pole + 1 < a.npole) fetch(pole + 1, nxt);
    const PoleCoef pc = a.coef[pole];
    const double2 al = pc.alpha;
    const double sre = pc.sig.x, sim = pc.sig.y;
    float2* gres = a.gres + ((long long)pole * a.w_pole + (long long)leaf * q2) * r + r0;
    for (int idx = threadIdx.x; idx < RR * q2; idx += blockDim.x) {
      const int k = idx / RR, jr = idx - k * RR;
      if (r0 + jr >= r) continue;
      const int i = k % q + 1, jj = k / q + 1;
      const double* mx = Mx + ((jj - 1) * q + (i - 1)) * p;
      const double* my = My + ((i - 1) * q + (jj - 1)) * p;
      double2 ky = make_double2(0.0, 0.0);
      for (int l = 0; l < p; ++l) {
        const double2 ux = U[(l + p * jj) * RR + jr];
        const double2 uy = U[(i + p * l) * RR + jr];
        ky.x += mx[l] * ux.x + my[l] * uy.x;
        ky.y += mx[l] * ux.y + my[l] * uy.y;
      }
      const double2 y = U[(i + p * jj) * RR + jr];
      // (K - s) y
      const double ar = ky.x - (sre * y.x - sim * y.y);
      const double ai = ky.y - (sre * y.y + sim * y.x);
      const double x1 = st[k * RR + jr], x2 = st[(q2 + k) * RR + jr];
      const double x3 = SW ? st[(2 * q2 + k) * RR + jr] : 0.0;
      const double gr = fma(pc.k1.x, x1, fma(pc.k2.x, x2, pc.k3.x * x3));
      const double gi = fma(pc.k1.y, x1, fma(pc.k2.y, x2, pc.k3.y * x3));
      gres[(long long)k * r + jr] = make_float2((float)(gr - ar), (float)(gi - ai));
    }
    // outward normal derivative at the edge slots: sx D[0 or p-1][.] along the row,
    // sy D[0 or p-1][.] along the column
    double2* dn = a.dn + ((long long)pole * a.e_pole + L.vec_off) * r + r0;
    for (int idx = threadIdx.x; idx < RR * L.e; idx += blockDim.x) {
      const int k = idx / RR, jr = idx - k * RR;
      if (r0 + jr >= r) continue;
      const int slot = k / q, t = k - slot * q;
      const int s = side_of_slot_r(L.side_mask, slot);
      const bool xn = s < 2, lo = (s == 0 || s == 2);
      const double* Dr = Ds + (lo ? 0 : (p - 1)) * p;
      const double sc = xn ? (lo ? -a.sx : a.sx) : (lo ? -a.sy : a.sy);
      double2 v = make_double2(0.0, 0.0);
      for (int l = 0; l < p; ++l) {
        const double2 u = xn ? U[(l + p * (t + 1)) * RR + jr] : U[((t + 1) + p * l) * RR + jr];
        v.x += Dr[l] * u.x;
        v.y += Dr[l] * u.y;
      }
      double2 out = make_double2(sc * v.x, sc * v.y);
      if constexpr (SW) {
        const int kw = a.slot_wall[L.vec_off + k];
        if (kw >= 0) {   // wall row: rhs_b - (a d_n y - f d_t y)
          // t = (-n2, n1): left -d_y, right +d_y, bottom +d_x, top -d_x
          const double tsc = (s == 0) ? -a.sy : (s == 1) ? a.sy : (s == 2) ? a.sx : -a.sx;
          double2 dt = make_double2(0.0, 0.0);
          for (int l = 0; l < q; ++l) {
            const int node = (s == 0) ? p * (l + 1) : (s == 1) ? (p - 1) + p * (l + 1)
                           : (s == 2) ? (l + 1) : (l + 1) + p * (p - 1);
            const double2 u = U[node * RR + jr];
            const double d = a.Dq[t * q + l];
            dt.x += d * u.x;
            dt.y += d * u.y;
          }
          dt.x *= tsc;
          dt.y *= tsc;
          const double ax = al.x * itau, ay = al.y * itau;
          const double* wv = a.wallv + (long long)(r0 + jr) * 2 * a.n_wall;
          const double nv = wv[kw] * itau * a.inv_c, tv = wv[a.n_wall + kw] * itau * a.inv_c;
          const double rr = ax * nv - a.f * tv - (ax * out.x - ay * out.y - a.f * dt.x);
          const double ri = ay * nv - (ax * out.y + ay * out.x - a.f * dt.y);
          out = make_double2(rr, ri);
        }
      }
      dn[(long long)k * r + jr] = out;
    }
  }
  if constexpr (SW) {   // first-sweep pole sums on the full grid
    const long long plane = (long long)a.n_leaf * pp;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = threadIdx.x + u * kBlock;
      if (idx < RR * pp) {
        const int node = idx / RR, jr = idx - node * RR;
        if (r0 + jr < r) {
          double* E = a.esum + (long long)(r0 + jr) * 3 * plane + (long long)leaf * pp + node;
          E[0] = e0[u];
          E[plane] = e1[u];
          E[2 * plane] = e2[u];
        }
      }
    }
  }
}

// Bytes of LDS for RR right-hand sides per block.
static size_t residual_lds(int p, int RR, int nsrc) {
  const int pp = p * p, q2 = (p - 2) * (p - 2);
  return sizeof(double) * (2 * (size_t)pp + 2 * (size_t)q2 * p + (size_t)nsrc * RR * q2) +
         sizeof(double2) * (size_t)RR * pp;
}

template <bool SW>
static hipError_t residual_t(const ResidualArgs& a, int n_leaf, hipStream_t s) {
  // right-hand sides per block: up to 32, within 56 KiB of LDS (two to
  // three blocks per CU), at least 1 (then up to 160 KiB); the grid values
  // of one pole are at most 8 per thread
  int RR = 32;
  while (RR > 1 && (RR / 2 >= a.nrhs || residual_lds(a.p, RR, a.nsrc) > 56 * 1024 ||
                    RR * a.p * a.p > 8 * kBlock))
    RR /= 2;
  const size_t lds = residual_lds(a.p, RR, a.nsrc);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_residual<SW>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int nrg = (a.nrhs + RR - 1) / RR;
  hipLaunchKernelGGL(k_residual<SW>, dim3(n_leaf * nrg), dim3(kBlock), lds, s, a, RR);
  return hipGetLastError();
}

hipError_t launch_residual(const ResidualArgs& a, int n_leaf, hipStream_t s) {
  if (a.esum) return residual_t<true>(a, n_leaf, s);
  return residual_t<false>(a, n_leaf, s);
}

}  // namespace hx
