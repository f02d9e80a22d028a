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
  const double* state;       // [rhs][field][n_int]
  long long rhs_stride;      // 2 * n_int
  int n_int;
  const PoleCoef* coef;
  double inv_tau, inv_tau2;
  const double* nrow;        // D[0][1..q] then D[p-1][1..q]
  double sx, sy;             // 2/hx, 2/hy
  int q;
  double2* w;                // [col][leaf][q*q]
  long long w_col_stride;
  double2* h;                // level-0 h: [col][sum of e]
  long long h_col_stride;
};

struct MergeArgs {
  const double2* ops;
  long long pole_stride;
  const BoxDesc* boxes;
  const int* idx;
  int ncol, nrhs, row_blocks;
  double2* child;            // level below: h (up) or u (down), [col][...]
  long long child_col_stride;
  double2* self;             // this level: h (up, written) or u (down, read)
  long long self_col_stride;
  double2* g3;               // this level's interface loads [col][...]
  long long g3_col_stride;
};

struct LeafDownArgs {
  const double2* ops;
  long long pole_stride;
  const LeafDesc* leaves;
  int ncol, nrhs, q;
  const double2* u;          // level-0 u: [col][sum of e]
  long long u_col_stride;
  double2* w;                // in: w, out: y
  long long w_col_stride;
};

struct PoleSumArgs {
  const LeafDesc* leaves;
  int npole, nrhs, q;
  const PoleCoef* coef;
  const double2* y;
  long long y_col_stride;
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

}  // namespace hx
