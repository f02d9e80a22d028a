// FP64 residual of the collocation equations (precision form).
//
// After the FP32 sweep every pole has a solution y0 on the element interiors
// and values u_e on the element edges.  Assembled on an element's full
// p x p grid (zero on the outer boundary), they give, in FP64,
//   * the residual of the PDE rows at the interior nodes (section 2.2):
//       res = g - (sx^2 Dx C^2 Dx + sy^2 Dy C^2 Dy - s) y,  g = (alpha u + tau v)/tau^2,
//   * the element's outward normal derivative at each of its edge slots;
//     the flux rows' residual at an interface node is minus the sum of its
//     two elements' values, added by the merge of the correction sweep.
// One block per (element, pole, group of RR right-hand sides); the grid
// values and first derivatives live in LDS.
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

__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs a, int RR) {
  extern __shared__ double sm[];
  const int p = a.p, q = a.q, q2 = q * q, pp = p * p;
  const int nrg = (a.nrhs + RR - 1) / RR;
  int rest = blockIdx.x;
  const int rg = rest % nrg; rest /= nrg;
  const int pole = rest % a.npole;
  const int leaf = rest / a.npole;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs;
  double* Ds = sm;
  double* cs = Ds + pp;
  double2* U = reinterpret_cast<double2*>(cs + pp);   // [RR][p*p]
  double2* UX = U + RR * pp;                          // x-derivative on interior rows
  double2* UY = UX + RR * pp;                         // y-derivative on interior columns
  for (int t = threadIdx.x; t < pp; t += blockDim.x) {
    Ds[t] = a.D[t];
    cs[t] = a.c2[(long long)L.elem * pp + t];
  }
  const float2* y0 = a.y0 + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
  const float2* ue = a.ue + ((long long)pole * a.e_pole + L.vec_off) * r;
  for (int idx = threadIdx.x; idx < RR * pp; idx += blockDim.x) {
    const int jr = idx / pp, node = idx - jr * pp;
    const int i = node % p, jj = node / p;
    const int rhs = rg * RR + jr;
    double2 v = make_double2(0.0, 0.0);
    if (rhs < r) {
      const bool ix = (i > 0 && i < p - 1), iy = (jj > 0 && jj < p - 1);
      if (ix && iy) {
        const float2 f = y0[(long long)((i - 1) + q * (jj - 1)) * r + rhs];
        v = make_double2(f.x, f.y);
      } else if (ix != iy) {  // non-corner edge node
        const int s = (i == 0) ? 0 : (i == p - 1) ? 1 : (jj == 0) ? 2 : 3;
        const int t = (s < 2) ? jj - 1 : i - 1;
        const int sl = slot_of_side(L.side_mask, s);
        if (sl >= 0) {
          const float2 f = ue[(long long)(sl * q + t) * r + rhs];
          v = make_double2(f.x, f.y);
        }
      }
    }
    U[jr * pp + node] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < RR * pp; idx += blockDim.x) {
    const int jr = idx / pp, node = idx - jr * pp;
    const int i = node % p, jj = node / p;
    const double2* Ur = U + jr * pp;
    double2 dx = make_double2(0.0, 0.0), dy = dx;
    if (jj > 0 && jj < p - 1)
      for (int l = 0; l < p; ++l) {
        const double d = Ds[i * p + l];
        dx.x += d * Ur[l + p * jj].x;
        dx.y += d * Ur[l + p * jj].y;
      }
    if (i > 0 && i < p - 1)
      for (int l = 0; l < p; ++l) {
        const double d = Ds[jj * p + l];
        dy.x += d * Ur[i + p * l].x;
        dy.y += d * Ur[i + p * l].y;
      }
    UX[jr * pp + node] = make_double2(a.sx * dx.x, a.sx * dx.y);
    UY[jr * pp + node] = make_double2(a.sy * dy.x, a.sy * dy.y);
  }
  __syncthreads();
  const double2 al = a.coef[pole].alpha;
  const double itau = 1.0 / a.tau;
  // s = (alpha / tau)^2
  const double sre = (al.x * al.x - al.y * al.y) * itau * itau;
  const double sim = 2.0 * al.x * al.y * itau * itau;
  float2* gres = a.gres + ((long long)pole * a.w_pole + (long long)leaf * q2) * r;
  for (int idx = threadIdx.x; idx < RR * q2; idx += blockDim.x) {
    const int jr = idx / q2, k = idx - jr * q2;
    const int rhs = rg * RR + jr;
    if (rhs >= r) continue;
    const int i = k % q + 1, jj = k / q + 1;
    const double2* UXr = UX + jr * pp;
    const double2* UYr = UY + jr * pp;
    double2 kx = make_double2(0.0, 0.0), ky = kx;
    for (int m = 0; m < p; ++m) {
      const double dxm = Ds[i * p + m] * cs[m + p * jj];
      kx.x += dxm * UXr[m + p * jj].x;
      kx.y += dxm * UXr[m + p * jj].y;
      const double dym = Ds[jj * p + m] * cs[i + p * m];
      ky.x += dym * UYr[i + p * m].x;
      ky.y += dym * UYr[i + p * m].y;
    }
    const double2 y = U[jr * pp + i + p * jj];
    // (K - s) y
    const double ar = a.sx * kx.x + a.sy * ky.x - (sre * y.x - sim * y.y);
    const double ai = a.sx * kx.y + a.sy * ky.y - (sre * y.y + sim * y.x);
    const double* st = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
    const double uu = st[k], vv = st[a.n_int + k];
    const double gr = fma(al.x * itau * itau, uu, vv * itau);
    const double gi = al.y * itau * itau * uu;
    gres[(long long)k * r + rhs] = make_float2((float)(gr - ar), (float)(gi - ai));
  }
  double2* dn = a.dn + ((long long)pole * a.e_pole + L.vec_off) * r;
  for (int idx = threadIdx.x; idx < RR * L.e; idx += blockDim.x) {
    const int jr = idx / L.e, k = idx - jr * L.e;
    const int rhs = rg * RR + jr;
    if (rhs >= r) continue;
    const int slot = k / q, t = k - slot * q;
    const int s = side_of_slot_r(L.side_mask, slot);
    double2 v;
    if (s == 0) v = UX[jr * pp + 0 + p * (t + 1)], v.x = -v.x, v.y = -v.y;
    else if (s == 1) v = UX[jr * pp + (p - 1) + p * (t + 1)];
    else if (s == 2) v = UY[jr * pp + (t + 1) + 0], v.x = -v.x, v.y = -v.y;
    else v = UY[jr * pp + (t + 1) + p * (p - 1)];
    dn[(long long)k * r + rhs] = v;
  }
}

hipError_t launch_residual(const ResidualArgs& a, int n_leaf, hipStream_t s) {
  const int pp = a.p * a.p;
  const int RR = a.p <= 16 ? 4 : 2;
  const size_t lds = sizeof(double) * 2 * pp + sizeof(double2) * 3 * (size_t)RR * pp;
  const int nrg = (a.nrhs + RR - 1) / RR;
  hipLaunchKernelGGL(k_residual, dim3(n_leaf * a.npole * nrg), dim3(kBlock), lds, s, a, RR);
  return hipGetLastError();
}

}  // namespace hx
