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

// Threads per block and grid items per thread: RR p^2 <= kPer kResBlock.
constexpr int kResBlock = 512;
constexpr int kPer = 4;

template <bool SW>
__device__ __forceinline__ void residual_body(const ResidualArgs& a, const int bid) {
  const int RR = a.RR;
  // Work items are rhs-fastest (RR is a power of two).  Each thread fetches
  // the same kPer grid items (node, rhs) for every pole, with offsets
  // computed once; the interior rows and edge slots look their node indices
  // up in small LDS tables.  The grid values are FP32 (as the sweep left
  // them) and widen to FP64 exactly where they are used.
  extern __shared__ double sm[];
  const int p = a.p, q = a.q, q2 = q * q, pp = p * p;
  const int lg = __ffs(RR) - 1;
  const int nrg = (a.nrhs + RR - 1) / RR;
  const int rg = bid % nrg;
  const int leaf = bid / nrg;
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
  float2* U = reinterpret_cast<float2*>(st + ns * RR * q2);     // grid values [p*p][RR]
  int* kij = reinterpret_cast<int*>(U + RR * pp);     // interior k -> i | jj << 8
  int* dmt = kij + q2;                                // edge slot k -> side | t << 2 | (wall+1) << 8
  for (int t = threadIdx.x; t < pp; t += blockDim.x) {
    Ds[t] = a.D[t];
    cs[t] = a.c2[(long long)L.elem * pp + t];
  }
  for (int k = threadIdx.x; k < q2; k += blockDim.x) kij[k] = (k % q + 1) | ((k / q + 1) << 8);
  for (int k = threadIdx.x; k < L.e; k += blockDim.x) {
    const int slot = k / q, t = k - slot * q;
    int kw = -1;
    if constexpr (SW) kw = a.slot_wall[L.vec_off + k];
    dmt[k] = side_of_slot_r(L.side_mask, slot) | (t << 2) | ((kw + 1) << 8);
  }
  for (int idx = threadIdx.x; idx < RR * ns * q2; idx += blockDim.x) {
    const int k = idx >> lg, jr = idx & (RR - 1);     // k < nsrc q^2: field-major
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
  // fetch offsets: >= 0 interior (y0), < -1 edge (ue at -2-off), -1 none
  int off[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + u * kResBlock;
    off[u] = -1;
    if (idx < RR * pp) {
      const int node = idx >> lg, jr = idx & (RR - 1);
      const int i = node % p, jj = node / p;
      if (r0 + jr < r) {
        const bool ix = (i > 0 && i < p - 1), iy = (jj > 0 && jj < p - 1);
        if (ix && iy) {
          off[u] = ((i - 1) + q * (jj - 1)) * r + jr;
        } else if (ix != iy) {  // non-corner edge node
          const int sd = (i == 0) ? 0 : (i == p - 1) ? 1 : (jj == 0) ? 2 : 3;
          const int t = (sd < 2) ? jj - 1 : i - 1;
          const int sl = slot_of_side(L.side_mask, sd);
          if (sl >= 0) off[u] = -2 - ((sl * q + t) * r + jr);
        }
      }
    }
  }
  const double itau = 1.0 / a.tau;
  const float2* y0b = a.y0 + (long long)leaf * q2 * r + r0;
  const float2* ueb = a.ue + (long long)L.vec_off * r + r0;
  auto fetch = [&](int pole, float2* buf) {
    const float2* y0 = y0b + (long long)pole * a.w_pole * r;
    const float2* ue = ueb + (long long)pole * a.e_pole * r;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      float2 v = make_float2(0.f, 0.f);
      if (off[u] >= 0) v = y0[off[u]];
      else if (off[u] < -1) v = ue[-2 - off[u]];
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
      const int idx = threadIdx.x + u * kResBlock;
      if (idx < RR * pp) {
        U[idx] = nxt[u];
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
    for (int idx = threadIdx.x; idx < RR * q2; idx += kResBlock) {
      const int jr = idx & (RR - 1), k = idx >> lg;
      if (r0 + jr >= r) continue;
      const int ij = kij[k];
      const int i = ij & 255, jj = ij >> 8;
      const double* mx = Mx + ((jj - 1) * q + (i - 1)) * p;
      const double* my = My + ((i - 1) * q + (jj - 1)) * p;
      const float2* ux = U + (p * jj) * RR + jr;      // row jj, stride RR
      const float2* uy = U + i * RR + jr;             // column i, stride p RR
      double2 ky = make_double2(0.0, 0.0);
      for (int l = 0; l < p; ++l) {
        const float2 a1 = ux[l * RR], a2 = uy[l * p * RR];
        ky.x += mx[l] * double(a1.x) + my[l] * double(a2.x);
        ky.y += mx[l] * double(a1.y) + my[l] * double(a2.y);
      }
      const float2 yf = U[(i + p * jj) * RR + jr];
      const double2 y = make_double2(yf.x, yf.y);
      // (K - sigma) y
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
    for (int idx = threadIdx.x; idx < RR * L.e; idx += kResBlock) {
      const int jr = idx & (RR - 1), k = idx >> lg;
      if (r0 + jr >= r) continue;
      const int dmk = dmt[k];
      const int sd = dmk & 3, t = (dmk >> 2) & 63;
      const bool xn = sd < 2, lo = (sd == 0 || sd == 2);
      const double* Dr = Ds + (lo ? 0 : (p - 1)) * p;
      const double sc = xn ? (lo ? -a.sx : a.sx) : (lo ? -a.sy : a.sy);
      const float2* ul = xn ? U + (p * (t + 1)) * RR + jr : U + (t + 1) * RR + jr;
      const int ls = xn ? RR : p * RR;
      double2 v = make_double2(0.0, 0.0);
      for (int l = 0; l < p; ++l) {
        const float2 uu = ul[l * ls];
        v.x += Dr[l] * double(uu.x);
        v.y += Dr[l] * double(uu.y);
      }
      double2 out = make_double2(sc * v.x, sc * v.y);
      if constexpr (SW) {
        const int kw = (dmk >> 8) - 1;
        if (kw >= 0) {   // wall row: rhs_b - (a d_n y - f d_t y)
          // t = (-n2, n1): left -d_y, right +d_y, bottom +d_x, top -d_x
          const double tsc = (sd == 0) ? -a.sy : (sd == 1) ? a.sy : (sd == 2) ? a.sx : -a.sx;
          // the side's q non-corner nodes: (0|p-1, l+1) or (l+1, 0|p-1)
          const float2* ut = (sd == 0) ? U + p * RR + jr
                           : (sd == 1) ? U + (2 * p - 1) * RR + jr
                           : (sd == 2) ? U + RR + jr : U + (p * (p - 1) + 1) * RR + jr;
          const int ts = xn ? p * RR : RR;
          double2 dt = make_double2(0.0, 0.0);
          for (int l = 0; l < q; ++l) {
            const float2 uu = ut[l * ts];
            const double d = a.Dq[t * q + l];
            dt.x += d * double(uu.x);
            dt.y += d * double(uu.y);
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
  if constexpr (SW) {   // first-sweep pole sums on the full grid, [leaf][3][p*p][rhs]
    double* E = a.esum + (long long)leaf * 3 * pp * r + r0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = threadIdx.x + u * kResBlock;
      if (idx < RR * pp) {
        const int node = idx >> lg, jr = idx & (RR - 1);
        if (r0 + jr < r) {
          E[(long long)node * r + jr] = e0[u];
          E[(long long)(pp + node) * r + jr] = e1[u];
          E[(long long)(2 * pp + node) * r + jr] = e2[u];
        }
      }
    }
  }
}

template <bool SW>
__global__ __launch_bounds__(kResBlock) void k_residual(ResidualArgs a) {
  residual_body<SW>(a, blockIdx.x);
}

template <bool SW>
__global__ __launch_bounds__(kResBlock) void k_residual_multi(Multi<ResidualArgs> m) {
  int i;
  const int bid = m.locate(blockIdx.x, i);
  const ResidualArgs a = m.args[i];
  residual_body<SW>(a, bid);
}

// Bytes of LDS for RR right-hand sides per block.
size_t residual_lds_bytes(int p, int RR, int nsrc) {
  const int pp = p * p, q2 = (p - 2) * (p - 2);
  return sizeof(double) * (2 * (size_t)pp + 2 * (size_t)q2 * p + (size_t)nsrc * RR * q2) +
         sizeof(float2) * (size_t)RR * pp + sizeof(int) * ((size_t)q2 + 4 * (p - 2));
}

// Right-hand sides per block: up to 32, within 56 KiB of LDS (two to three
// blocks per CU), at least 1 (then up to 160 KiB); the grid values of one
// pole are at most kPer per thread.
int residual_rr(const ResidualArgs& a) {
  int RR = 32;
  while (RR > 1 && (RR / 2 >= a.nrhs || residual_lds_bytes(a.p, RR, a.nsrc) > 56 * 1024 ||
                    RR * a.p * a.p > kPer * kResBlock))
    RR /= 2;
  return RR;
}

template <bool SW>
static hipError_t allow_residual_lds(size_t lds, bool multi) {
  if (lds <= 65536) return hipSuccess;
  const void* f = multi ? reinterpret_cast<const void*>(&k_residual_multi<SW>)
                        : reinterpret_cast<const void*>(&k_residual<SW>);
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_residual_one(const ResidualArgs& a, int blocks, bool sw, size_t lds, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  const hipError_t e = sw ? allow_residual_lds<true>(lds, false) : allow_residual_lds<false>(lds, false);
  if (e != hipSuccess) return e;
  if (sw) hipLaunchKernelGGL(k_residual<true>, dim3(blocks), dim3(kResBlock), lds, s, a);
  else hipLaunchKernelGGL(k_residual<false>, dim3(blocks), dim3(kResBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_residual_multi(const Multi<ResidualArgs>& m, int blocks, bool sw, size_t lds,
                                 hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  const hipError_t e = sw ? allow_residual_lds<true>(lds, true) : allow_residual_lds<false>(lds, true);
  if (e != hipSuccess) return e;
  if (sw) hipLaunchKernelGGL(k_residual_multi<true>, dim3(blocks), dim3(kResBlock), lds, s, m);
  else hipLaunchKernelGGL(k_residual_multi<false>, dim3(blocks), dim3(kResBlock), lds, s, m);
  return hipGetLastError();
}

}  // namespace hx
