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

__global__ __launch_bounds__(kBlock) void k_sw_prep(SwPrepArgs a) {
  __shared__ double Dq[(kMaxP - 2) * (kMaxP - 2)];
  const int leaf = blockIdx.x / a.nrhs;
  const int rhs = blockIdx.x - leaf * a.nrhs;
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

__global__ __launch_bounds__(kBlock) void k_sw_wall(SwWallArgs a) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
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
  // bottom (0,-1),(1,0); top (0,1),(-1,0)
  double nv, tv;
  if (side == 0) { nv = -e1; tv = -e2; }
  else if (side == 1) { nv = e1; tv = e2; }
  else if (side == 2) { nv = -e2; tv = e1; }
  else { nv = e2; tv = -e1; }
  a.out[(long long)rhs * 2 * a.n_wall + k] = nv;
  a.out[(long long)rhs * 2 * a.n_wall + a.n_wall + k] = tv;
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

template <class T>
__global__ __launch_bounds__(kBlock) void k_sw_post(SwPostArgs<T> a) {
  extern __shared__ double smem[];
  const int p = a.p, q = a.q, q2 = q * q, pp = p * p;
  const int leaf = blockIdx.x / a.nrhs;
  const int rhs = blockIdx.x - leaf * a.nrhs;
  const LeafDesc L = a.leaves[leaf];
  const int r = a.nrhs;
  double* Ds = smem;                  // p x p
  double* E = Ds + pp;                // [3][p*p]: E0, E1, E2 on the full grid
  for (int t = threadIdx.x; t < pp; t += blockDim.x) Ds[t] = a.D[t];
  // precision form: start from the first sweep's sums (FP64)
  const long long plane = (long long)a.n_leaf * pp;
  const double* es = a.esum ? a.esum + (long long)rhs * 3 * plane + (long long)leaf * pp : nullptr;
  for (int t = threadIdx.x; t < 3 * pp; t += blockDim.x) {
    const int fld = t / pp, node = t - fld * pp;
    E[t] = es ? es[fld * plane + node] : 0.0;
  }
  __syncthreads();
  // interior nodes: sum over poles of the leaf sweep's solutions
  for (int k = threadIdx.x; k < q2; k += blockDim.x) {
    const int node = (k % q + 1) + p * (k / q + 1);
    double s0 = 0, s1 = 0, s2 = 0;
    for (int pole = 0; pole < a.npole; ++pole) {
      const typename Cplx<T>::type y =
          a.y[((long long)pole * a.y_pole + (long long)leaf * q2 + k) * r + rhs];
      const SwCoef c = a.coef[pole];
      s0 += c.c0.x * double(y.x) - c.c0.y * double(y.y);
      s1 += c.c1.x * double(y.x) - c.c1.y * double(y.y);
      s2 += c.c2.x * double(y.x) - c.c2.y * double(y.y);
    }
    E[node] += s0;
    E[pp + node] += s1;
    E[2 * pp + node] += s2;
  }
  // edge nodes (all four sides carry exterior values)
  for (int k = threadIdx.x; k < L.e; k += blockDim.x) {
    const int slot = k / q, t = k - slot * q;
    int s = -1, seen = -1;
    for (int m = 0; m < 4; ++m)
      if ((L.side_mask >> m) & 1)
        if (++seen == slot) { s = m; break; }
    const int node = (s == 0) ? p * (t + 1) : (s == 1) ? (p - 1) + p * (t + 1)
                   : (s == 2) ? (t + 1) : (t + 1) + p * (p - 1);
    double s0 = 0, s1 = 0, s2 = 0;
    for (int pole = 0; pole < a.npole; ++pole) {
      const typename Cplx<T>::type y =
          a.ue[((long long)pole * a.e_pole + L.vec_off + k) * r + rhs];
      const SwCoef c = a.coef[pole];
      s0 += c.c0.x * double(y.x) - c.c0.y * double(y.y);
      s1 += c.c1.x * double(y.x) - c.c1.y * double(y.y);
      s2 += c.c2.x * double(y.x) - c.c2.y * double(y.y);
    }
    E[node] += s0;
    E[pp + node] += s1;
    E[2 * pp + node] += s2;
  }
  __syncthreads();
  double* st = a.state + rhs * a.rhs_stride + (long long)L.elem * q2;
  for (int k = threadIdx.x; k < q2; k += blockDim.x) {
    const int i = k % q + 1, j = k / q + 1;
    double e1x = 0, e1y = 0, e2x = 0, e2y = 0;
    for (int m = 0; m < p; ++m) {
      const double dx = Ds[i * p + m], dy = Ds[j * p + m];
      e1x += dx * E[pp + m + p * j];
      e2x += dx * E[2 * pp + m + p * j];
      e1y += dy * E[pp + i + p * m];
      e2y += dy * E[2 * pp + i + p * m];
    }
    e1x *= a.sx; e2x *= a.sx; e1y *= a.sy; e2y *= a.sy;
    const double v1 = st[k], v2 = st[a.n_int + k];
    const double c = a.c, f = a.f;
    st[k] = c * e1x - c * f * e2y - (a.beta1 * v1 - f * a.beta2 * v2) * a.inv_tau;
    st[a.n_int + k] = c * e1y + c * f * e2x - (a.beta1 * v2 + f * a.beta2 * v1) * a.inv_tau;
    st[2 * a.n_int + k] = E[(i + p * j)];
  }
}

hipError_t launch_sw_prep(const SwPrepArgs& a, int n_leaf, hipStream_t s) {
  hipLaunchKernelGGL(k_sw_prep, dim3(n_leaf * a.nrhs), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sw_wall(const SwWallArgs& a, hipStream_t s) {
  const long long n = (long long)a.n_wall * a.nrhs;
  hipLaunchKernelGGL(k_sw_wall, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sw_root_form(const SwRootFormArgs& a, int chunk, hipStream_t s) {
  const long long nn = (long long)a.n * a.n;
  long long bx = (nn + kBlock - 1) / kBlock;
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_sw_root_form, dim3((unsigned)bx, chunk), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sw_post(const SwPostArgs<T>& a, int n_leaf, hipStream_t s) {
  const size_t lds = sizeof(double) * 4 * (size_t)a.p * a.p;
  hipLaunchKernelGGL((k_sw_post<T>), dim3(n_leaf * a.nrhs), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

template hipError_t launch_sw_post<double>(const SwPostArgs<double>&, int, hipStream_t);
template hipError_t launch_sw_post<float>(const SwPostArgs<float>&, int, hipStream_t);

}  // namespace hx
