// Kernel argument blocks and launchers of the hpsexp library.
#pragma once

#include "hx_internal.h"

namespace hx {

constexpr int kMaxQ2 = (kMaxP - 2) * (kMaxP - 2);

// ---- solve stage (apply) ----------------------------------------------------

struct LeafUpArgs {
  const double2* ops;        // operator block of pole 0; pole k at ops + k*pole_stride
  long long pole_stride;
  const LeafDesc* leaves;
  int ncol, nrhs;            // columns = poles * nrhs
  const double* state;       // source fields X: [rhs][field][n_int]
  long long rhs_stride;      // fields * n_int
  int n_int;
  int nsrc;                  // source fields used (2 or 3)
  const PoleCoef* coef;
  double inv_tau, inv_tau2;
  const double* nrow;        // D[0][1..q] then D[p-1][1..q]
  double sx, sy;             // 2/hx, 2/hy
  int q;
  double2* w;                // [pole][leaf][q*q][rhs]
  long long w_pole;          // nodes per pole: n_leaf * q*q
  double2* h;                // level-0 h: [pole][sum of e][rhs]
  long long h_pole;
};

struct MergeArgs {
  const double2* ops;
  long long pole_stride;
  const BoxDesc* boxes;
  const int* idx;
  int ncol, nrhs, row_blocks;
  double2* child;            // level below: h (up) or u (down), [pole][node][rhs]
  long long child_pole;      // nodes per pole in that level
  double2* self;             // this level: h (up, written) or u (down, read)
  long long self_pole;
  double2* g3;               // this level's interface loads [pole][node][rhs]
  long long g3_pole;
};

struct LeafDownArgs {
  const double2* ops;
  long long pole_stride;
  const LeafDesc* leaves;
  int ncol, nrhs, q;
  const double2* u;          // level-0 u: [pole][sum of e][rhs]
  long long u_pole;
  double2* w;                // in: w, out: y   [pole][leaf][q*q][rhs]
  long long w_pole;
};

struct PoleSumArgs {
  const LeafDesc* leaves;
  int npole, nrhs, q;
  const PoleCoef* coef;
  const double2* y;          // [pole][leaf][q*q][rhs]
  long long y_pole;
  double* state;
  long long rhs_stride;
  int n_int;
  double beta, inv_tau;
};

hipError_t launch_leaf_up(const LeafUpArgs& a, int n_leaf, hipStream_t s);
hipError_t launch_merge_up(const MergeArgs& a, int n_box, int max_n3, hipStream_t s);
hipError_t launch_merge_down(const MergeArgs& a, int n_box, int max_x, hipStream_t s);
hipError_t launch_leaf_down(const LeafDownArgs& a, int n_leaf, hipStream_t s);
hipError_t launch_pole_sum(const PoleSumArgs& a, int n_leaf, hipStream_t s);

// ---- solve stage, many right-hand sides (matrix cores) -----------------------

// Several instances in one launch: instance i owns the blocks
// [first[i], first[i+1]) and its arguments are args[i] (device tables).
template <class A>
struct Multi {
  const A* args;
  const int* first;   // n + 1 entries
  int n;
  __device__ int locate(int b, int& i) const {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first[mid] <= b) lo = mid;
      else hi = mid - 1;
    }
    i = lo;
    return b - first[lo];
  }
};

// Right-hand-side tiles of 16 * nt columns.
inline int mm_tiles(int nrhs, int nt) { return (nrhs + 16 * nt - 1) / (16 * nt); }

template <class T> struct Cplx;
template <> struct Cplx<double> { typedef double2 type; };
template <> struct Cplx<float> { typedef float2 type; };

template <class T>
struct MmLeafUpArgs {
  const typename Cplx<T>::type* ops;
  long long pole_stride;
  const LeafDesc* leaves;
  int npole, nrhs, q;
  const double* state;       // source fields X: [rhs][field][n_int]
  long long rhs_stride;
  int n_int;
  int nsrc;
  const PoleCoef* coef;
  double inv_tau, inv_tau2;
  const double* nrow;
  double sx, sy;
  typename Cplx<T>::type* w;   // [pole][leaf][q*q][rhs]
  long long w_pole;
  typename Cplx<T>::type* h;   // [pole][sum of e][rhs]
  long long h_pole;
  // precision form, correction sweep: right-hand side taken from the
  // residual [pole][leaf][q*q][rhs] instead of the state (null: state)
  const typename Cplx<T>::type* gin;
  int w_lds;                 // keep the w tile in LDS for h (the launch's LDS allows it)
  int pole_group;            // poles walked by one block (blocks: leaves x tiles x groups)
  int x_lds;                 // stage the source fields in LDS once per block (else read per pole)
};

template <class T>
struct MmMergeArgs {
  const typename Cplx<T>::type* ops;
  long long pole_stride;
  const BoxDesc* boxes;
  const int* idx;
  int npole, nrhs, row_groups;
  typename Cplx<T>::type* child;
  long long child_pole;
  typename Cplx<T>::type* self;
  long long self_pole;
  typename Cplx<T>::type* g3;
  long long g3_pole;
  // precision form, correction sweep: flux-jump residual from the element
  // normal derivatives dn [pole][sum of e][rhs], FP64 because the two
  // elements' values nearly cancel (null: none)
  const double2* dn;
  long long dn_pole;
  // upward pass: poles per block (>= 1); a block walks poles
  // [g G, (g + 1) G) of its box, row group and RHS tile (downward: 1)
  int pole_group;
};

// Two merge levels in one launch, l and l + 1 (l >= 1): a block holds one
// level-(l+1) box, one pole and one RHS tile; the level-l vectors between
// the two merges stay in LDS.  Upward: child = level l-1 h, self = level
// l+1 h; downward: child = level l-1 u, self = level l+1 u.
template <class T>
struct MmMerge2Args {
  const typename Cplx<T>::type* ops;
  long long pole_stride;
  const BoxDesc* lo;   // level l boxes
  const BoxDesc* hi;   // level l + 1 boxes
  const int* idx;
  int npole, nrhs;
  typename Cplx<T>::type* child;
  long long child_pole;
  typename Cplx<T>::type* self;
  long long self_pole;
  typename Cplx<T>::type* g3_lo;
  long long g3_lo_pole;
  typename Cplx<T>::type* g3_hi;
  long long g3_hi_pole;
  const double2* dn;   // upward correction sweep, as in MmMergeArgs
  long long dn_pole;
};

template <class T>
struct MmLeafDownArgs {
  const typename Cplx<T>::type* ops;
  long long pole_stride;
  const LeafDesc* leaves;
  int npole, nrhs, q, row_groups;
  const typename Cplx<T>::type* u;
  long long u_pole;
  typename Cplx<T>::type* w;
  long long w_pole;
  // pole sum (fused variant only)
  const PoleCoef* coef;
  double* state;
  long long rhs_stride;
  int n_int;
  double beta, inv_tau;
  // precision form: y0 = first-sweep solution; the unfused variant writes
  // y = w - S u_e there, the fused variant sums y0 + w - S u_e (null: unused)
  typename Cplx<T>::type* y0;
};

// ---- shallow water -----------------------------------------------------------

struct SwPrepArgs {
  const double* state;       // [rhs][3][n_int]: v1, v2, eta
  double* prep;              // [rhs][3][n_int]: eta, div v, curl v
  long long rhs_stride;
  int n_int, nrhs, q;
  const double* Dq;          // q x q interior-line differentiation (reference)
  double sx, sy;
};

struct SwWallArgs {
  const double* state;
  long long rhs_stride;
  int n_int, nrhs, q, n_wall;
  const int4* wall;          // per root exterior slot: element, side, node along the side
  const double* w_lo;        // extrapolation weights to the low / high end of a line
  const double* w_hi;
  double* out;               // [rhs][2][n_wall]: n.v, t.v
};

struct SwRootFormArgs {
  const double2* T;          // root DtN of each chunk pole
  long long T_stride;
  const double* Dt;          // tangential derivative on the wall slots (n x n)
  int n;
  double f;
  const double2* a;          // a = alpha/tau per chunk pole
  double2* G;                // [chunk][n*n]
};

template <class T>
struct SwPostArgs {
  const LeafDesc* leaves;
  int npole, nrhs, p, q;
  const double* D;           // p x p
  const SwCoef* coef;
  const typename Cplx<T>::type* y;   // interior solutions [pole][leaf][q*q][rhs]
  long long y_pole;
  const typename Cplx<T>::type* ue;  // edge values, level-0 u [pole][sum e][rhs]
  long long e_pole;
  double* state;
  long long rhs_stride;
  int n_int;
  double sx, sy, c, f, beta1, beta2, inv_tau;
  const double* esum;        // precision form: first-sweep sums [leaf][3][p*p][rhs] (null: none)
  int n_leaf;
  int RR;                    // right-hand sides per block (set by sw_post_rr)
};

template <class T>
struct SwRootArgs {
  const typename Cplx<T>::type* ops;   // Q of pole k at ops + k*pole_stride + q_off
  long long pole_stride, q_off;
  int n, npole, nrhs, row_groups;
  const PoleCoef* coef;
  double inv_tau, inv_c, f;
  const double* wall;                  // [rhs][2][n]: n.v, t.v
  const typename Cplx<T>::type* h;     // root h [pole][n][rhs]
  typename Cplx<T>::type* u;           // root u (wall values) [pole][n][rhs]
  // precision form, correction sweep: the wall-row residual at level-0 slot
  // wall_info[k].w of pole p, rw[(p * rw_pole + slot) * nrhs + rhs] (null: none)
  const double2* rw;
  long long rw_pole;
  const int4* wall_info;
};

hipError_t launch_sw_root_form(const SwRootFormArgs& a, int chunk, hipStream_t s);
hipError_t launch_sw_prep_multi(const Multi<SwPrepArgs>& m, int blocks, hipStream_t s);
hipError_t launch_sw_wall_multi(const Multi<SwWallArgs>& m, int blocks, hipStream_t s);
template <class T>
hipError_t launch_sw_post_multi(const Multi<SwPostArgs<T>>& m, int blocks, size_t lds, hipStream_t s);
int sw_post_rr(int p, int nrhs);
size_t sw_post_lds_bytes(int p, int RR);

// FP64 residual of the collocation equations for the precision form.
struct ResidualArgs {
  const LeafDesc* leaves;
  int npole, nrhs, p, q;
  const double* c2;          // [elem][p*p]
  const double* D;           // p x p row-major
  double sx, sy, tau;
  const PoleCoef* coef;
  const double* state;
  long long rhs_stride;
  int n_int;
  const float2* y0;          // first-sweep interior solution [pole][leaf][q*q][rhs]
  long long w_pole;
  const float2* ue;          // first-sweep edge values (level-0 u) [pole][sum e][rhs]
  long long e_pole;
  float2* gres;              // residual of the interior rows, same layout as y0
  double2* dn;               // outward normal derivative at the edge slots, as ue (FP64);
                             // shallow water: the wall-row residual at wall slots
  int nsrc;                  // source fields of g (state is the source array)
  // shallow water only
  int n_leaf;
  const int* slot_wall;      // per level-0 slot: wall index, -1 for interface slots
  const double* wallv;       // [rhs][2][n_wall]: n.v, t.v
  int n_wall;
  const double* Dq;          // q x q interior-line differentiation
  double f, inv_c;
  const SwCoef* swc;
  double* esum;              // first-sweep pole sums E0, E1, E2 [leaf][3][p*p][rhs]
  int RR;                    // right-hand sides per block (set by residual_rr)
};
int residual_rr(const ResidualArgs& a);                       // RR for one instance
size_t residual_lds_bytes(int p, int RR, int nsrc);
hipError_t launch_residual_multi(const Multi<ResidualArgs>& m, int blocks, bool sw, size_t lds,
                                 hipStream_t s);

// Multi-instance variants: one launch over the blocks of every instance in
// the table, all with the same tile count nt (1 or 2) and LDS bytes.
template <class T> hipError_t launch_leaf_up_mm_multi(const Multi<MmLeafUpArgs<T>>& m, int blocks, int nt, bool xl, size_t lds, hipStream_t s);
template <class T> hipError_t launch_merge_up_mm_multi(const Multi<MmMergeArgs<T>>& m, int blocks, int nt, int wv, hipStream_t s);
template <class T> hipError_t launch_merge2_up_mm_multi(const Multi<MmMerge2Args<T>>& m, int blocks, int nt, size_t lds, hipStream_t s);
template <class T> hipError_t launch_merge2_down_mm_multi(const Multi<MmMerge2Args<T>>& m, int blocks, int nt, size_t lds, hipStream_t s);
template <class T> hipError_t launch_merge2_up_mm_one(const MmMerge2Args<T>& a, int blocks, int nt, size_t lds, hipStream_t s);
template <class T> hipError_t launch_merge2_down_mm_one(const MmMerge2Args<T>& a, int blocks, int nt, size_t lds, hipStream_t s);
// LDS bytes of a fused two-level block for the given box sizes.
template <class T> size_t merge2_up_lds_bytes(int nt, int child_rows, int mid_rows, int stage_rows);
template <class T> size_t merge2_down_lds_bytes(int nt, int rows);
template <class T> hipError_t launch_merge_down_mm_multi(const Multi<MmMergeArgs<T>>& m, int blocks, int nt, int wv, hipStream_t s);
template <class T> hipError_t launch_leaf_down_mm_multi(const Multi<MmLeafDownArgs<T>>& m, int blocks, int nt, hipStream_t s);
template <class T> hipError_t launch_leaf_down_sum_mm_multi(const Multi<MmLeafDownArgs<T>>& m, int blocks, int nt, hipStream_t s);
template <class T> hipError_t launch_sw_root_mm_multi(const Multi<SwRootArgs<T>>& m, int blocks, int nt, hipStream_t s);
// The same launches for one instance, arguments by value.
template <class T> hipError_t launch_leaf_up_mm_one(const MmLeafUpArgs<T>& a, int blocks, int nt, size_t lds, hipStream_t s);
template <class T> hipError_t launch_merge_up_mm_one(const MmMergeArgs<T>& a, int blocks, int nt, int wv, hipStream_t s);
template <class T> hipError_t launch_merge_down_mm_one(const MmMergeArgs<T>& a, int blocks, int nt, int wv, hipStream_t s);
template <class T> hipError_t launch_leaf_down_mm_one(const MmLeafDownArgs<T>& a, int blocks, int nt, hipStream_t s);
template <class T> hipError_t launch_leaf_down_sum_mm_one(const MmLeafDownArgs<T>& a, int blocks, int nt, hipStream_t s);
template <class T> hipError_t launch_sw_root_mm_one(const SwRootArgs<T>& a, int blocks, int nt, hipStream_t s);
hipError_t launch_residual_one(const ResidualArgs& a, int blocks, bool sw, size_t lds, hipStream_t s);
hipError_t launch_sw_prep_one(const SwPrepArgs& a, int blocks, hipStream_t s);
hipError_t launch_sw_wall_one(const SwWallArgs& a, int blocks, hipStream_t s);
template <class T>
hipError_t launch_sw_post_one(const SwPostArgs<T>& a, int blocks, size_t lds, hipStream_t s);
// LDS bytes of the leaf upward kernel (above 64 KiB the launcher raises the
// kernel's dynamic LDS limit).
template <class T> size_t leaf_up_lds_bytes(int q, int nt, bool with_w, int nsrc_staged);

// nt = right-hand-side tiles of 16 per block (1 or 2)

// ---- build stage ------------------------------------------------------------

struct LeafAssembleArgs {
  const double* c2;          // [elem][p*p]
  const double* D;           // p x p, row-major
  int p, q, n_leaf, chunk;
  double sx, sy;
  const double2* sigma;      // per chunk pole
  const LeafDesc* leaves;
  double2* A;                // [chunk][leaf][q2*q2]
  double2* ops;              // operator block of the chunk's first pole
  long long pole_stride;
};

struct LeafDtnArgs {
  const double* D;
  int p, q, n_leaf, chunk;
  double sx, sy;
  const LeafDesc* leaves;
  const double2* ops;        // [W | S] of the chunk's first pole
  long long pole_stride;
  double2* T;                // [chunk][sum of e^2]
  long long T_stride;
  const long long* T_off;    // per leaf
};

struct MergeGatherArgs {
  const BoxDesc* boxes;
  const int* idx;
  int chunk;
  const double2* Tc;         // children T: [chunk][...]
  long long Tc_stride;
  const long long* Tc_off;   // per box of the level below
  double2* M;                // [chunk][sum n3^2]
  long long M_stride;
  const long long* M_off;
  double2* V;                // [chunk][sum ext*n3]
  long long V_stride;
  const long long* V_off;
  double2* Tp;               // [chunk][sum ext^2]
  long long Tp_stride;
  const long long* Tp_off;
  double2* ops;              // Z of the chunk's first pole
  long long pole_stride;
};

hipError_t launch_leaf_assemble(const LeafAssembleArgs& a, hipStream_t s);
hipError_t launch_leaf_dtn(const LeafDtnArgs& a, hipStream_t s);
hipError_t launch_merge_gather(const MergeGatherArgs& a, int n_box, hipStream_t s);
hipError_t launch_nonfinite_check(const double* x, long long n, int* flag, hipStream_t s);
hipError_t launch_pack_f32(const double2* src, float2* dst, long long n, hipStream_t s);
hipError_t launch_eye(double2* X, int n, hipStream_t s);

}  // namespace hx
