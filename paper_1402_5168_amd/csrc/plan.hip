// Host side of the hpsexp C-ABI: plans, merge trees, validation, arena
// layout, the build stage (rocSOLVER / rocBLAS for the dense factorisations)
// and the step (kernel sequence, replayed from a hipGraph).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "hpsexp.h"
#include "hx_kernels.h"

namespace {

using cd = std::complex<double>;
using hx::BoxDesc;
using hx::LeafDesc;
using hx::PoleCoef;
using hx::SwCoef;

thread_local std::string g_last_error;

hx_status fail(hx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = std::string(hx_status_str(st)) + ": " + buf;
  return st;
}

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(HX_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                  __FILE__, __LINE__);                                                \
  } while (0)

#define RB_OK(expr)                                                                   \
  do {                                                                                \
    rocblas_status s_ = (expr);                                                       \
    if (s_ != rocblas_status_success)                                                 \
      return fail(HX_EDEVICE, "%s failed: rocblas status %d (%s:%d)", #expr, (int)s_, \
                  __FILE__, __LINE__);                                                \
  } while (0)

#define HX_TRY(expr)                  \
  do {                                \
    hx_status st_ = (expr);           \
    if (st_ != HX_OK) return st_;     \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
constexpr size_t kArgsMax = 256;   // bytes of the largest argument block
constexpr size_t kTabSlot = 512;   // table bytes reserved per recorded stage
bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Chebyshev-Lobatto differentiation matrix on ascending nodes
// x_k = -cos(k pi / N), N = p-1 (section 2.2), row-major D[i*p + j].
std::vector<double> cheb_diff(int p) {
  const int N = p - 1;
  std::vector<double> D(p * p, 0.0);
  auto c = [&](int k) { return (k == 0 || k == N) ? 2.0 : 1.0; };
  for (int i = 0; i < p; ++i) {
    double rowsum = 0.0;
    for (int j = 0; j < p; ++j) {
      if (i == j) continue;
      // x_i - x_j = 2 sin((i+j) pi / 2N) sin((i-j) pi / 2N)
      const double dx = 2.0 * std::sin((i + j) * M_PI / (2.0 * N)) *
                        std::sin((i - j) * M_PI / (2.0 * N));
      const double sgn = ((i + j) % 2) ? -1.0 : 1.0;
      D[i * p + j] = c(i) / c(j) * sgn / dx;
      rowsum += D[i * p + j];
    }
    D[i * p + i] = -rowsum;
  }
  return D;
}

struct Level {
  std::vector<BoxDesc> boxes;
  int total_ext = 0, total_n3 = 0, max_ext = 0, max_n3 = 0, max_x = 0;
  // device offsets (bytes inside the arena)
  size_t d_boxes = 0, d_h = 0, d_u = 0, d_g3 = 0;
};

// Stages of a step in launch order (the recorder's order key; the tuned
// choices of an instance are kept per stage).
enum StageOrder : int { O_PREP, O_LEAF_UP, O_MERGE_UP, O_ROOT, O_MERGE_DOWN, O_LEAF_DOWN, O_RESIDUAL, O_POST };

struct Instance {
  hx_mesh mesh{};
  int q = 0, q2 = 0, n_leaf = 0, npole = 0, nrhs = 0, ncol = 0, M = 0;
  double tau = 0.0, delta = 0.0, beta = 0.0;
  std::vector<double> c2;
  std::vector<cd> alpha, b;                 // m = -M..M
  std::vector<LeafDesc> leaves;
  std::vector<Level> levels;                // levels[0] = leaves (boxes empty)
  std::vector<int> idx;
  std::vector<PoleCoef> coef;
  std::vector<double> nrow;
  long long pole_stride = 0;                // complex elements per pole block
  long long leaf_ops = 0, merge_ops = 0;    // complex elements per pole
  double max_abs_R = 0.0, fit_X = 0.0, sum_abs_b = 0.0;
  int tune_nt[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // per stage: right-hand-side tiles (0: default)
  int tune_wv[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // merge stages: 1 = one-wave blocks at every level
  int tune_xl = 0;                          // upward elements: 2 = never stage the sources
  int tune_pg[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // merge stages: 1 = one pole per block
  int tune_fuse[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // merge stages: 1 = fused pairs of low levels
  bool fp32 = false;                        // precision form: FP32 operators and sweeps
  // shallow water: wall nodes are exterior unknowns up to the root
  bool sw = false;
  int nfield = 2;
  double f = 0.0, cw = 1.0;                 // Coriolis frequency, sqrt(gH)
  double beta1 = 0.0, beta2 = 0.0;          // sum_m b a/s, sum_m b/s
  int n_wall = 0;
  long long q_off = 0;                      // root wall system Q inside a pole block
  std::vector<int4> wall;                   // per root exterior slot: element, side, node
  std::vector<double> Dt;                   // tangential derivative on the wall slots
  std::vector<double> Dq, w_lo, w_hi;       // interior-line differentiation and end weights
  std::vector<SwCoef> swcoef;
  std::vector<int> slot_wall;               // per level-0 slot: wall index or -1
  size_t d_esum = 0, d_slotw = 0;           // precision form only
  size_t d_prep = 0, d_wallv = 0, d_wall = 0, d_Dq = 0, d_wlo = 0, d_whi = 0, d_swc = 0;
  // arena layout (byte offsets)
  size_t d_ops = 0, d_w = 0, d_leaves = 0, d_idx = 0, d_coef = 0, d_nrow = 0, end = 0;
  size_t d_y0 = 0, d_gres = 0, d_dn = 0, d_c2 = 0, d_D = 0;  // precision form only
  size_t cbytes() const { return fp32 ? sizeof(float2) : sizeof(double2); }
};

// One fused launch of the batched instances: a stage kind and tile count,
// its instances' argument table and block offsets inside the arena.
struct Group {
  int kind, nt, wv, cls, n;
  long long blocks;
  size_t lds, args_off, first_off;
};

}  // namespace

struct hx_plan {
  int device = 0;
  int precision = HX_FP64;
  unsigned flags = 0;
  std::vector<Instance> inst;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  bool built = false;
  // graph cache
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<double*> graph_states;
  hipStream_t graph_stream = nullptr;
  int* d_flag = nullptr;  // inside the arena
  size_t d_flag_off = 0;
  // stage tables of the batched instances (fused launches)
  size_t d_tab = 0, tab_bytes = 0;
  bool tab_ready = false;
  std::vector<double*> tab_states;
  std::vector<Group> groups;
  std::vector<unsigned char> tab_blob;
};

namespace {

// Many right-hand sides go through the matrix-core kernels unless the plan
// asks for one pass per right-hand side (the unbatched reference); the
// precision form always does.
bool batched(const hx_plan* plan, const Instance& I) {
  return I.fp32 || I.sw || (I.nrhs > 1 && !(plan->flags & HX_FLAG_UNBATCHED));
}

// ---- rational function checks (eqs. RM_prop1 and RM_prop2) ----------------

cd R_eval(const Instance& I, double x) {
  const cd z(0.0, x);
  cd s = 0.0;
  for (int k = 0; k < I.npole * 2 - 1; ++k) s += I.b[k] / (z - I.alpha[k]);
  return s;
}

void check_fit(Instance& I) {
  double mx = 0.0;
  auto probe = [&](double x) { mx = std::max(mx, std::abs(R_eval(I, x))); };
  for (int k = 0; k <= 80000; ++k) probe(-400.0 + k * 0.01);
  for (int k = 0; k <= 4000; ++k) {
    const double x = 400.0 * std::pow(1e7 / 400.0, k / 4000.0);
    probe(x);
    probe(-x);
  }
  I.max_abs_R = mx;
  // largest X with |R(ix) - e^{ix}| <= delta on [-X, X] (grid step 1e-3)
  double X = 0.0;
  for (int k = 0;; ++k) {
    const double x = k * 1e-3;
    const double e1 = std::abs(R_eval(I, x) - std::exp(cd(0.0, x)));
    const double e2 = std::abs(R_eval(I, -x) - std::exp(cd(0.0, -x)));
    if (std::max(e1, e2) > I.delta || x > 1e5) break;
    X = x;
  }
  I.fit_X = X;
  double sb = 0.0;
  for (auto& v : I.b) sb += std::abs(v);
  I.sum_abs_b = sb;
}

// ---- merge tree --------------------------------------------------------------

struct TBox {
  int x0, y0, w, h;
  std::vector<int> ext;  // global interface node ids (outer boundary pruned)
};

void build_tree(Instance& I) {
  const int nex = I.mesh.nex, ney = I.mesh.ney, q = I.q;
  const int n_vert = (nex - 1) * ney * q;
  auto vnode = [&](int vx, int ey, int t) { return (vx + (nex - 1) * ey) * q + t; };
  auto hnode = [&](int ex, int hy, int t) { return n_vert + (ex + nex * hy) * q + t; };
  const int n_iface = n_vert + nex * (ney - 1) * q;
  // wall nodes (shallow water only): left, right, bottom, top walls
  auto wnode = [&](int side, int k, int t) {
    const int off = side == 0 ? 0 : side == 1 ? ney * q : side == 2 ? 2 * ney * q
                                                                    : 2 * ney * q + nex * q;
    return n_iface + off + k * q + t;
  };
  const int n_nodes = n_iface + (I.sw ? 2 * (nex + ney) * q : 0);
  std::vector<int4> wall_of(std::max(n_nodes, 1), make_int4(-1, -1, -1, 0));

  std::vector<TBox> cur;
  I.leaves.clear();
  I.levels.clear();
  I.levels.emplace_back();
  long long op = 0;
  int vec = 0;
  // the two element-edge slots (level-0 vector positions) of each interface node
  std::vector<int> slot_a(std::max(n_nodes, 1), -1), slot_b(std::max(n_nodes, 1), -1);
  for (int ey = 0; ey < ney; ++ey)
    for (int ex = 0; ex < nex; ++ex) {
      TBox b{ex, ey, 1, 1, {}};
      int mask = 0;
      const int el = ex + nex * ey;
      auto add_wall = [&](int side, int k) {
        for (int t = 0; t < q; ++t) {
          const int id = wnode(side, k, t);
          wall_of[id] = make_int4(el, side, t, 0);
          b.ext.push_back(id);
        }
      };
      if (ex > 0) { mask |= 1; for (int t = 0; t < q; ++t) b.ext.push_back(vnode(ex - 1, ey, t)); }
      else if (I.sw) { mask |= 1; add_wall(0, ey); }
      if (ex < nex - 1) { mask |= 2; for (int t = 0; t < q; ++t) b.ext.push_back(vnode(ex, ey, t)); }
      else if (I.sw) { mask |= 2; add_wall(1, ey); }
      if (ey > 0) { mask |= 4; for (int t = 0; t < q; ++t) b.ext.push_back(hnode(ex, ey - 1, t)); }
      else if (I.sw) { mask |= 4; add_wall(2, ex); }
      if (ey < ney - 1) { mask |= 8; for (int t = 0; t < q; ++t) b.ext.push_back(hnode(ex, ey, t)); }
      else if (I.sw) { mask |= 8; add_wall(3, ex); }
      for (size_t k = 0; k < b.ext.size(); ++k) {
        int& sl = slot_a[b.ext[k]] < 0 ? slot_a[b.ext[k]] : slot_b[b.ext[k]];
        sl = vec + (int)k;
      }
      LeafDesc L{};
      L.op_off = op;
      L.vec_off = vec;
      L.e = (int)b.ext.size();
      L.side_mask = mask;
      L.elem = ex + nex * ey;
      I.leaves.push_back(L);
      op += align_up((size_t)I.q2 * (I.q2 + L.e), 8);
      vec += L.e;
      cur.push_back(std::move(b));
    }
  I.leaf_ops = op;
  I.levels[0].total_ext = vec;
  for (auto& L : I.leaves) I.levels[0].max_ext = std::max(I.levels[0].max_ext, L.e);

  std::vector<int> pos(std::max(n_nodes, 1), -1);
  int nbx = nex, nby = ney;
  I.idx.clear();
  while (nbx * nby > 1) {
    const bool in_x = nbx > 1 && (cur[0].w <= cur[0].h || nby == 1);
    const int nbx2 = in_x ? nbx / 2 : nbx, nby2 = in_x ? nby : nby / 2;
    Level lev;
    std::vector<TBox> next;
    int vec_off = 0, g3_off = 0;
    const Level& below = I.levels.back();
    std::vector<int> below_vec;
    if (I.levels.size() == 1)
      for (auto& L : I.leaves) below_vec.push_back(L.vec_off);
    else
      for (auto& B : below.boxes) below_vec.push_back(B.vec_off);
    for (int by = 0; by < nby2; ++by)
      for (int bx = 0; bx < nbx2; ++bx) {
        const int ia = in_x ? (2 * bx + nbx * by) : (bx + nbx * (2 * by));
        const int ib = in_x ? (2 * bx + 1 + nbx * by) : (bx + nbx * (2 * by + 1));
        const TBox& A = cur[ia];
        const TBox& Bb = cur[ib];
        for (size_t k = 0; k < Bb.ext.size(); ++k) pos[Bb.ext[k]] = (int)k;
        std::vector<int> s1, s3, i1, i3a, s2, i2, i3b;
        for (size_t k = 0; k < A.ext.size(); ++k) {
          if (pos[A.ext[k]] >= 0) s3.push_back(A.ext[k]);
          else { s1.push_back(A.ext[k]); i1.push_back((int)k); }
        }
        for (size_t k = 0; k < Bb.ext.size(); ++k) pos[Bb.ext[k]] = -1;
        std::sort(s3.begin(), s3.end());
        // positions of the interface nodes in a and b
        for (size_t k = 0; k < A.ext.size(); ++k) pos[A.ext[k]] = (int)k;
        for (int id : s3) i3a.push_back(pos[id]);
        for (size_t k = 0; k < A.ext.size(); ++k) pos[A.ext[k]] = -1;
        for (size_t k = 0; k < Bb.ext.size(); ++k) pos[Bb.ext[k]] = (int)k;
        for (int id : s3) i3b.push_back(pos[id]);
        for (size_t k = 0; k < Bb.ext.size(); ++k) pos[Bb.ext[k]] = -1;
        for (int id : s3) pos[id] = 0;
        for (size_t k = 0; k < Bb.ext.size(); ++k)
          if (pos[Bb.ext[k]] < 0) { s2.push_back(Bb.ext[k]); i2.push_back((int)k); }
        for (int id : s3) pos[id] = -1;

        BoxDesc D{};
        D.n1 = (int)s1.size();
        D.n2 = (int)s2.size();
        D.n3 = (int)s3.size();
        D.a_box = ia;
        D.b_box = ib;
        D.a_vec = below_vec[ia];
        D.b_vec = below_vec[ib];
        D.vec_off = vec_off;
        D.g3_off = g3_off;
        D.idx_off = (int)I.idx.size();
        I.idx.insert(I.idx.end(), i1.begin(), i1.end());
        I.idx.insert(I.idx.end(), i2.begin(), i2.end());
        I.idx.insert(I.idx.end(), i3a.begin(), i3a.end());
        I.idx.insert(I.idx.end(), i3b.begin(), i3b.end());
        D.j_off = (int)I.idx.size();
        for (int id : s3) I.idx.push_back(slot_a[id]);
        for (int id : s3) I.idx.push_back(slot_b[id]);
        const long long ext = D.n1 + D.n2;
        D.op_off = op;
        op += align_up((size_t)(D.n3 * (ext + D.n3) + ext * D.n3), 8);
        vec_off += (int)ext;
        g3_off += D.n3;
        lev.max_ext = std::max(lev.max_ext, (int)ext);
        lev.max_n3 = std::max(lev.max_n3, D.n3);
        lev.max_x = std::max(lev.max_x, (int)ext + D.n3);
        lev.boxes.push_back(D);

        TBox P{A.x0, A.y0, in_x ? A.w * 2 : A.w, in_x ? A.h : A.h * 2, {}};
        P.ext = s1;
        P.ext.insert(P.ext.end(), s2.begin(), s2.end());
        next.push_back(std::move(P));
      }
    lev.total_ext = vec_off;
    lev.total_n3 = g3_off;
    I.levels.push_back(std::move(lev));
    cur.swap(next);
    nbx = nbx2;
    nby = nby2;
  }
  // shallow water: the wall slots in the root's exterior order, their
  // tangential derivative and the root wall system Q (n_wall^2) per pole
  I.wall.clear();
  if (I.sw) {
    const std::vector<int>& rext = cur[0].ext;
    I.n_wall = (int)rext.size();
    I.slot_wall.assign(std::max(I.levels[0].total_ext, 1), -1);
    for (int id : rext) {
      int4 wi = wall_of[id];
      wi.w = slot_a[id];                     // the wall node's level-0 slot
      I.slot_wall[wi.w] = (int)I.wall.size();
      I.wall.push_back(wi);
    }
    const int n = I.n_wall;
    I.Dt.assign((size_t)n * n, 0.0);
    std::map<std::pair<int, int>, std::vector<int>> seg;   // (element, side) -> slots by t
    for (int k = 0; k < n; ++k) {
      auto& v = seg[{I.wall[k].x, I.wall[k].y}];
      if ((int)v.size() < q) v.resize(q, -1);
      v[I.wall[k].z] = k;
    }
    const double sx = 2.0 * nex / (I.mesh.x1 - I.mesh.x0), sy = 2.0 * ney / (I.mesh.y1 - I.mesh.y0);
    for (auto& kv : seg) {
      const int side = kv.first.second;
      // t = (-n2, n1): left -d_y, right +d_y, bottom +d_x, top -d_x
      const double sg = (side == 0 || side == 3) ? -1.0 : 1.0;
      const double sc = side < 2 ? sy : sx;
      for (int t1 = 0; t1 < q; ++t1)
        for (int t2 = 0; t2 < q; ++t2)
          I.Dt[(size_t)kv.second[t1] + (size_t)kv.second[t2] * n] = sg * sc * I.Dq[t1 * q + t2];
    }
    I.q_off = op;
    op += align_up((size_t)n * n, 8);
  }
  I.merge_ops = op - I.leaf_ops;
  I.pole_stride = align_up((size_t)op, 16);
}

// Stages an instance records per step on the matrix-core path.
size_t stage_count(const Instance& I) {
  const size_t nl = I.levels.size(), passes = I.fp32 ? 2 : 1;
  size_t n = passes * (1 + 2 * (nl - 1) + 1 + (I.sw ? 1 : 0));
  if (I.fp32) n += 1;                 // residual
  if (I.sw) n += 3;                   // sources, wall values, velocity recovery
  return n;
}

void layout_arena(hx_plan* plan) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  plan->d_flag_off = take(sizeof(int));
  size_t n_stages = 0;
  for (auto& I : plan->inst)
    if (I.fp32 || I.sw || I.nrhs > 1) n_stages += stage_count(I);
  plan->tab_bytes = n_stages * kTabSlot + kAlign;
  plan->d_tab = take(plan->tab_bytes);
  for (auto& I : plan->inst) {
    const size_t cb = I.cbytes();
    I.d_ops = take(cb * (size_t)I.pole_stride * I.npole);
    I.d_w = take(cb * (size_t)I.ncol * I.n_leaf * I.q2);
    for (size_t l = 0; l < I.levels.size(); ++l) {
      Level& L = I.levels[l];
      L.d_h = take(cb * (size_t)I.ncol * L.total_ext);
      L.d_u = take(cb * (size_t)I.ncol * L.total_ext);
      L.d_g3 = take(cb * (size_t)I.ncol * L.total_n3);
      L.d_boxes = take(sizeof(BoxDesc) * L.boxes.size());
    }
    if (I.sw) {
      I.d_prep = take(sizeof(double) * 3 * (size_t)I.nrhs * I.n_leaf * I.q2);
      I.d_wallv = take(sizeof(double) * 2 * (size_t)I.nrhs * I.n_wall);
      I.d_wall = take(sizeof(int4) * I.wall.size());
      I.d_Dq = take(sizeof(double) * I.Dq.size());
      I.d_wlo = take(sizeof(double) * I.w_lo.size());
      I.d_whi = take(sizeof(double) * I.w_hi.size());
      I.d_swc = take(sizeof(SwCoef) * I.swcoef.size());
      if (I.fp32) {
        I.d_esum = take(sizeof(double) * 3 * (size_t)I.nrhs * I.n_leaf * I.mesh.p * I.mesh.p);
        I.d_slotw = take(sizeof(int) * I.slot_wall.size());
      }
    }
    if (I.fp32) {
      I.d_y0 = take(cb * (size_t)I.ncol * I.n_leaf * I.q2);
      I.d_gres = take(cb * (size_t)I.ncol * I.n_leaf * I.q2);
      I.d_dn = take(sizeof(double2) * (size_t)I.ncol * I.levels[0].total_ext);
      I.d_c2 = take(sizeof(double) * I.c2.size());
    }
    if (I.sw || I.fp32) I.d_D = take(sizeof(double) * I.mesh.p * I.mesh.p);
    I.d_leaves = take(sizeof(LeafDesc) * I.leaves.size());
    I.d_idx = take(sizeof(int) * I.idx.size());
    I.d_coef = take(sizeof(PoleCoef) * I.coef.size());
    I.d_nrow = take(sizeof(double) * I.nrow.size());
    I.end = off;
  }
  plan->arena_bytes = off;
}

// Build workspace layout for a chunk of `ch` poles of one instance.
struct WsLayout {
  size_t A = 0, T0 = 0, T1 = 0, ipiv = 0, info = 0, ptr = 0, c2 = 0, D = 0, sigma = 0,
         toff = 0, ops64 = 0, Dt = 0, sa = 0, total = 0;
  long long sizeA = 0, sizeT = 0, sizeIpiv = 0, sizeInfo = 0, sizePtr = 0, n_off = 0;
};

WsLayout ws_layout(const Instance& I, int ch) {
  WsLayout w;
  w.sizeA = (long long)I.n_leaf * I.q2 * I.q2;
  w.sizeIpiv = (long long)I.n_leaf * I.q2;
  w.sizeInfo = I.n_leaf;
  long long t0 = 0;
  for (auto& L : I.leaves) t0 += (long long)L.e * L.e;
  w.sizeT = t0;
  w.n_off = (long long)I.leaves.size();
  for (size_t l = 1; l < I.levels.size(); ++l) {
    long long m = 0, v = 0, t = 0, pv = 0;
    for (auto& B : I.levels[l].boxes) {
      const long long ext = B.n1 + B.n2;
      m += (long long)B.n3 * B.n3;
      v += ext * B.n3;
      t += ext * ext;
      pv += B.n3;
    }
    w.sizeA = std::max(w.sizeA, m + v);
    w.sizeT = std::max(w.sizeT, t);
    w.sizeIpiv = std::max(w.sizeIpiv, pv);
    w.sizeInfo = std::max(w.sizeInfo, (long long)I.levels[l].boxes.size());
    w.n_off = std::max(w.n_off, (long long)I.levels[l].boxes.size());
  }
  if (I.sw) {   // root wall system G = a T_root - f D_t, and its pivots
    w.sizeA = std::max(w.sizeA, (long long)I.n_wall * I.n_wall);
    w.sizeIpiv = std::max(w.sizeIpiv, (long long)I.n_wall);
    w.sizeInfo = std::max(w.sizeInfo, 1LL);
  }
  w.sizePtr = 6 * w.sizeInfo;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  w.A = take(sizeof(double2) * (size_t)w.sizeA * ch);
  w.T0 = take(sizeof(double2) * (size_t)w.sizeT * ch);
  w.T1 = take(sizeof(double2) * (size_t)w.sizeT * ch);
  w.ipiv = take(sizeof(int) * (size_t)w.sizeIpiv * ch);
  w.info = take(sizeof(int) * (size_t)w.sizeInfo * ch);
  w.ptr = take(sizeof(void*) * (size_t)w.sizePtr * ch);
  w.c2 = take(sizeof(double) * I.c2.size());
  w.D = take(sizeof(double) * I.mesh.p * I.mesh.p);
  w.sigma = take(sizeof(double2) * ch);
  w.toff = take(sizeof(long long) * 4 * (size_t)std::max<long long>(w.n_off, 1));
  if (I.sw) {
    w.Dt = take(sizeof(double) * I.Dt.size());
    w.sa = take(sizeof(double2) * ch);
  }
  if (I.fp32) w.ops64 = take(sizeof(double2) * (size_t)I.pole_stride * ch);
  w.total = off;
  return w;
}

// ---- validation ---------------------------------------------------------------

hx_status validate_add(const hx_mesh* m, const hx_coeffs* c, double tau, double delta,
                       const hx_rational* r, int nrhs) {
  if (!m || !c || !r) return fail(HX_EINVAL, "null mesh, coeffs or rational");
  if (!is_pow2(m->nex) || !is_pow2(m->ney))
    return fail(HX_EINVAL, "nex=%d and ney=%d must be powers of two", m->nex, m->ney);
  if (m->p < 4 || m->p > hx::kMaxP) return fail(HX_EINVAL, "p=%d outside [4, %d]", m->p, hx::kMaxP);
  if (!(m->x1 > m->x0) || !(m->y1 > m->y0) || !std::isfinite(m->x0 + m->x1 + m->y0 + m->y1))
    return fail(HX_EINVAL, "empty or non-finite domain");
  if ((long long)m->nex * m->ney > (1LL << 22)) return fail(HX_EINVAL, "mesh too large");
  if (c->kind == HX_WAVE_DIRICHLET) {
    if (!c->c2) return fail(HX_EINVAL, "c2 is null");
    const long long n = (long long)m->nex * m->ney * m->p * m->p;
    for (long long k = 0; k < n; ++k)
      if (!(std::isfinite(c->c2[k]) && c->c2[k] > 0.0))
        return fail(HX_EINVAL, "c2[%lld] = %g is not finite and positive", k, c->c2[k]);
  } else if (c->kind == HX_SW_SLIP) {
    if (!std::isfinite(c->f)) return fail(HX_EINVAL, "f must be finite");
    if (!(c->gH > 0.0) || !std::isfinite(c->gH)) return fail(HX_EINVAL, "gH must be finite and > 0");
  } else {
    return fail(HX_EINVAL, "unsupported problem kind %d", c->kind);
  }
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(HX_EINVAL, "tau must be finite and > 0");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(HX_EINVAL, "delta must be finite and > 0");
  if (r->npoles < 1 || r->npoles % 2 == 0 || r->npoles > 4001)
    return fail(HX_EINVAL, "npoles=%d must be odd, 1..4001", r->npoles);
  if (!r->alpha || !r->b) return fail(HX_EINVAL, "alpha or b is null");
  const int M = (r->npoles - 1) / 2;
  for (int k = 0; k < 2 * r->npoles; ++k)
    if (!std::isfinite(r->alpha[k]) || !std::isfinite(r->b[k]))
      return fail(HX_EINVAL, "non-finite pole or residue");
  for (int m = 0; m <= M; ++m) {
    const cd ap(r->alpha[2 * (M + m)], r->alpha[2 * (M + m) + 1]);
    const cd am(r->alpha[2 * (M - m)], r->alpha[2 * (M - m) + 1]);
    const cd bp(r->b[2 * (M + m)], r->b[2 * (M + m) + 1]);
    const cd bm(r->b[2 * (M - m)], r->b[2 * (M - m) + 1]);
    if (std::abs(ap - std::conj(am)) > 1e-12 * std::max(1.0, std::abs(ap)))
      return fail(HX_EINVAL, "alpha_{-%d} != conj(alpha_%d)", m, m);
    if (std::abs(bp - std::conj(bm)) > 1e-12 * std::max(1.0, std::abs(bp)))
      return fail(HX_EINVAL, "b_{-%d} != conj(b_%d)", m, m);
    if (ap.real() == 0.0) return fail(HX_EINVAL, "Re(alpha_%d) = 0 (pole on the spectrum)", m);
  }
  if (nrhs < 1 || nrhs > 4096) return fail(HX_EINVAL, "nrhs=%d outside [1, 4096]", nrhs);
  return HX_OK;
}

// ---- build ---------------------------------------------------------------------

struct Build {
  hx_plan* plan;
  rocblas_handle rb = nullptr;
  hipStream_t s = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
};

template <class T>
T* wsp(const Build& B, size_t off) { return reinterpret_cast<T*>(B.ws + off); }

// Host-to-device copy that completes before returning (the host staging
// vectors of the build are reused right after).
hx_status upload(const Build& B, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return HX_OK;
  HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, B.s));
  HIP_OK(hipStreamSynchronize(B.s));
  return HX_OK;
}

hx_status check_info(const Build& B, const WsLayout& W, long long n, const char* what, int level) {
  std::vector<int> info(n);
  HIP_OK(hipMemcpyAsync(info.data(), B.ws + W.info, sizeof(int) * n, hipMemcpyDeviceToHost, B.s));
  HIP_OK(hipStreamSynchronize(B.s));
  for (long long k = 0; k < n; ++k)
    if (info[k] != 0)
      return fail(HX_ESINGULAR, "%s system %lld at level %d is singular (info %d)", what, k,
                  level, info[k]);
  return HX_OK;
}

// Shallow water: the root's wall values solve (a T_root - f D_t) eta_b =
// rhs_b - a h_root (the oblique slip condition); Q = (a T_root - f D_t)^{-1}
// is stored per pole.  Tc holds the root DtN map of every chunk pole.
hx_status build_root_walls(Build& B, Instance& I, const WsLayout& W, double2* ops, size_t Tc,
                           int p0, int ch) {
  const int n = I.n_wall;
  if (n == 0) return HX_OK;
  std::vector<double2> av(ch);
  for (int j = 0; j < ch; ++j) {
    const cd ap = I.alpha[I.M + p0 + j] / I.tau;
    av[j] = make_double2(ap.real(), ap.imag());
  }
  HX_TRY(upload(B, B.ws + W.sa, av.data(), sizeof(double2) * ch));
  HX_TRY(upload(B, B.ws + W.Dt, I.Dt.data(), sizeof(double) * I.Dt.size()));
  hx::SwRootFormArgs rf{};
  rf.T = wsp<double2>(B, Tc);
  rf.T_stride = W.sizeT;
  rf.Dt = wsp<double>(B, W.Dt);
  rf.n = n;
  rf.f = I.f;
  rf.a = wsp<double2>(B, W.sa);
  rf.G = wsp<double2>(B, W.A);
  HIP_OK(hx::launch_sw_root_form(rf, ch, B.s));
  std::vector<void*> ptrs;
  for (int j = 0; j < ch; ++j) ptrs.push_back(wsp<double2>(B, W.A) + (long long)j * n * n);
  for (int j = 0; j < ch; ++j) ptrs.push_back(ops + (long long)j * I.pole_stride + I.q_off);
  HX_TRY(upload(B, B.ws + W.ptr, ptrs.data(), sizeof(void*) * ptrs.size()));
  for (int j = 0; j < ch; ++j) HIP_OK(hx::launch_eye(ops + (long long)j * I.pole_stride + I.q_off, n, B.s));
  using P = rocblas_double_complex* const*;
  void** dptr = wsp<void*>(B, W.ptr);
  int* ipiv = wsp<int>(B, W.ipiv);
  int* info = wsp<int>(B, W.info);
  RB_OK(rocsolver_zgetrf_batched(B.rb, n, n, (P)dptr, n, ipiv, n, info, ch));
  RB_OK(rocsolver_zgetrs_batched(B.rb, rocblas_operation_none, n, n, (P)dptr, n, ipiv, n,
                                 (P)(dptr + ch), n, ch));
  return check_info(B, W, ch, "root wall", (int)I.levels.size() - 1);
}

hx_status build_chunk(Build& B, Instance& I, const WsLayout& W, int p0, int ch) {
  // FP64 operators of this chunk: straight into the arena, or into the
  // workspace first when the arena holds FP32 operators
  double2* ops = I.fp32 ? wsp<double2>(B, W.ops64)
                        : reinterpret_cast<double2*>(B.plan->arena + I.d_ops) + (long long)p0 * I.pole_stride;
  const int q2 = I.q2;
  const double sx = 2.0 * I.mesh.nex / (I.mesh.x1 - I.mesh.x0);
  const double sy = 2.0 * I.mesh.ney / (I.mesh.y1 - I.mesh.y0);
  std::vector<double2> sig(ch);
  for (int j = 0; j < ch; ++j) {
    const cd ap = I.alpha[I.M + p0 + j] / I.tau;
    const cd s = I.sw ? (ap * ap + I.f * I.f) / (I.cw * I.cw) : ap * ap;
    sig[j] = make_double2(s.real(), s.imag());
  }
  HX_TRY(upload(B, B.ws + W.sigma, sig.data(), sizeof(double2) * ch));

  // leaf systems: assemble, factor, solve [W | S] in place, DtN maps
  hx::LeafAssembleArgs la{};
  la.c2 = wsp<double>(B, W.c2);
  la.D = wsp<double>(B, W.D);
  la.p = I.mesh.p;
  la.q = I.q;
  la.n_leaf = I.n_leaf;
  la.chunk = ch;
  la.sx = sx;
  la.sy = sy;
  la.sigma = wsp<double2>(B, W.sigma);
  la.leaves = reinterpret_cast<const LeafDesc*>(B.plan->arena + I.d_leaves);
  la.A = wsp<double2>(B, W.A);
  la.ops = ops;
  la.pole_stride = I.pole_stride;
  HIP_OK(hx::launch_leaf_assemble(la, B.s));

  // group leaves by edge count (same right-hand side width)
  std::map<int, std::vector<int>> cls;
  for (int l = 0; l < I.n_leaf; ++l) cls[I.leaves[l].e].push_back(l);
  std::vector<void*> ptrs;
  struct Call { int e, n; size_t pa, pb; long long piv; };
  std::vector<Call> calls;
  long long piv = 0;
  for (auto& kv : cls) {
    Call c{kv.first, (int)kv.second.size() * ch, ptrs.size(), 0, piv};
    for (int j = 0; j < ch; ++j)
      for (int l : kv.second) ptrs.push_back(wsp<double2>(B, W.A) + ((long long)j * I.n_leaf + l) * q2 * q2);
    c.pb = ptrs.size();
    for (int j = 0; j < ch; ++j)
      for (int l : kv.second) ptrs.push_back(ops + (long long)j * I.pole_stride + I.leaves[l].op_off);
    piv += (long long)c.n;
    calls.push_back(c);
  }
  HX_TRY(upload(B, B.ws + W.ptr, ptrs.data(), sizeof(void*) * ptrs.size()));
  void** dptr = wsp<void*>(B, W.ptr);
  for (auto& c : calls) {
    auto A = reinterpret_cast<rocblas_double_complex* const*>(dptr + c.pa);
    auto R = reinterpret_cast<rocblas_double_complex* const*>(dptr + c.pb);
    int* ipiv = wsp<int>(B, W.ipiv) + c.piv * q2;
    int* info = wsp<int>(B, W.info) + c.piv;
    RB_OK(rocsolver_zgetrf_batched(B.rb, q2, q2, A, q2, ipiv, q2, info, c.n));
    RB_OK(rocsolver_zgetrs_batched(B.rb, rocblas_operation_none, q2, q2 + c.e, A, q2, ipiv, q2, R,
                                   q2, c.n));
  }
  HX_TRY(check_info(B, W, piv, "element", 0));

  // T offsets per leaf, then the DtN maps
  std::vector<long long> toff(I.n_leaf);
  long long t = 0;
  for (int l = 0; l < I.n_leaf; ++l) { toff[l] = t; t += (long long)I.leaves[l].e * I.leaves[l].e; }
  long long* d_toff = wsp<long long>(B, W.toff);
  HX_TRY(upload(B, d_toff, toff.data(), sizeof(long long) * toff.size()));
  hx::LeafDtnArgs ld{};
  ld.D = la.D;
  ld.p = I.mesh.p;
  ld.q = I.q;
  ld.n_leaf = I.n_leaf;
  ld.chunk = ch;
  ld.sx = sx;
  ld.sy = sy;
  ld.leaves = la.leaves;
  ld.ops = ops;
  ld.pole_stride = I.pole_stride;
  ld.T = wsp<double2>(B, W.T0);
  ld.T_stride = W.sizeT;
  ld.T_off = d_toff;
  HIP_OK(hx::launch_leaf_dtn(ld, B.s));

  size_t Tc = W.T0, Tp = W.T1;
  std::vector<long long> child_off = toff;
  for (size_t lv = 1; lv < I.levels.size(); ++lv) {
    const Level& L = I.levels[lv];
    const int nb = (int)L.boxes.size();
    std::vector<long long> moff(nb), voff(nb), poff(nb);
    long long m = 0, v = 0, pt = 0;
    for (int k = 0; k < nb; ++k) {
      const BoxDesc& D = L.boxes[k];
      const long long ext = D.n1 + D.n2;
      moff[k] = m; m += (long long)D.n3 * D.n3;
      voff[k] = v; v += ext * D.n3;
      poff[k] = pt; pt += ext * ext;
    }
    // offsets: [child T | M | V | Tpar] in one upload
    std::vector<long long> offs;
    offs.insert(offs.end(), child_off.begin(), child_off.end());
    offs.insert(offs.end(), moff.begin(), moff.end());
    offs.insert(offs.end(), voff.begin(), voff.end());
    offs.insert(offs.end(), poff.begin(), poff.end());
    long long* d_offs = wsp<long long>(B, W.toff);
    HX_TRY(upload(B, d_offs, offs.data(), sizeof(long long) * offs.size()));
    double2* Mbuf = wsp<double2>(B, W.A);
    double2* Vbuf = Mbuf + m * ch;
    hx::MergeGatherArgs mg{};
    mg.boxes = reinterpret_cast<const BoxDesc*>(B.plan->arena + L.d_boxes);
    mg.idx = reinterpret_cast<const int*>(B.plan->arena + I.d_idx);
    mg.chunk = ch;
    mg.Tc = wsp<double2>(B, Tc);
    mg.Tc_stride = W.sizeT;
    mg.Tc_off = d_offs;
    mg.M = Mbuf;
    mg.M_stride = m;
    mg.M_off = d_offs + child_off.size();
    mg.V = Vbuf;
    mg.V_stride = v;
    mg.V_off = d_offs + child_off.size() + nb;
    mg.Tp = wsp<double2>(B, Tp);
    mg.Tp_stride = W.sizeT;
    mg.Tp_off = d_offs + child_off.size() + 2 * nb;
    mg.ops = ops;
    mg.pole_stride = I.pole_stride;
    HIP_OK(hx::launch_merge_gather(mg, nb, B.s));

    // classes of identical shapes
    std::map<std::tuple<int, int, int>, std::vector<int>> mc;
    for (int k = 0; k < nb; ++k) mc[{L.boxes[k].n1, L.boxes[k].n2, L.boxes[k].n3}].push_back(k);
    ptrs.clear();
    struct MCall { int n1, n2, n3, n; size_t pM, pZ, pV, pX, pY, pT; long long piv; };
    std::vector<MCall> mcalls;
    long long mpiv = 0;
    for (auto& kv : mc) {
      MCall c{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
              (int)kv.second.size() * ch, 0, 0, 0, 0, 0, 0, mpiv};
      const long long ext = c.n1 + c.n2;
      auto push = [&](auto fn) {
        const size_t at = ptrs.size();
        for (int j = 0; j < ch; ++j)
          for (int k : kv.second) ptrs.push_back(fn(j, k));
        return at;
      };
      c.pM = push([&](int j, int k) -> void* { return Mbuf + (long long)j * m + moff[k]; });
      c.pZ = push([&](int j, int k) -> void* { return ops + (long long)j * I.pole_stride + L.boxes[k].op_off; });
      c.pV = push([&](int j, int k) -> void* { return Vbuf + (long long)j * v + voff[k]; });
      c.pX = push([&](int j, int k) -> void* {
        return ops + (long long)j * I.pole_stride + L.boxes[k].op_off + (long long)c.n3 * ext; });
      c.pY = push([&](int j, int k) -> void* {
        return ops + (long long)j * I.pole_stride + L.boxes[k].op_off + (long long)c.n3 * (ext + c.n3); });
      c.pT = push([&](int j, int k) -> void* { return wsp<double2>(B, Tp) + (long long)j * W.sizeT + poff[k]; });
      mpiv += c.n;
      mcalls.push_back(c);
    }
    HX_TRY(upload(B, B.ws + W.ptr, ptrs.data(), sizeof(void*) * ptrs.size()));
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0}, mone{-1.0, 0.0};
    long long ipiv_off = 0;
    for (auto& c : mcalls) {
      using P = rocblas_double_complex* const*;
      using CP = const rocblas_double_complex* const*;
      const int ext = c.n1 + c.n2;
      int* ipiv = wsp<int>(B, W.ipiv) + ipiv_off;
      int* info = wsp<int>(B, W.info) + c.piv;
      ipiv_off += (long long)c.n * c.n3;
      RB_OK(rocsolver_zgetrf_batched(B.rb, c.n3, c.n3, (P)(dptr + c.pM), c.n3, ipiv, c.n3, info, c.n));
      RB_OK(rocsolver_zgetrs_batched(B.rb, rocblas_operation_none, c.n3, ext + c.n3, (P)(dptr + c.pM),
                                     c.n3, ipiv, c.n3, (P)(dptr + c.pZ), c.n3, c.n));
      if (ext == 0) continue;
      // Y = V X
      RB_OK(rocblas_zgemm_batched(B.rb, rocblas_operation_none, rocblas_operation_none, ext, c.n3,
                                  c.n3, &one, (CP)(dptr + c.pV), ext, (CP)(dptr + c.pX), c.n3, &zero,
                                  (P)(dptr + c.pY), ext, c.n));
      // T_par = diag(T11a, T22b) - V X B
      if (lv + 1 < I.levels.size() || I.sw)
        RB_OK(rocblas_zgemm_batched(B.rb, rocblas_operation_none, rocblas_operation_none, ext, ext,
                                    c.n3, &mone, (CP)(dptr + c.pV), ext, (CP)(dptr + c.pZ), c.n3, &one,
                                    (P)(dptr + c.pT), ext, c.n));
    }
    HX_TRY(check_info(B, W, mpiv, "merge", (int)lv));
    std::swap(Tc, Tp);
    child_off = poff;
  }
  if (I.sw) HX_TRY(build_root_walls(B, I, W, ops, Tc, p0, ch));
  if (I.fp32) {
    float2* dst = reinterpret_cast<float2*>(B.plan->arena + I.d_ops) + (long long)p0 * I.pole_stride;
    HIP_OK(hx::launch_pack_f32(ops, dst, (long long)ch * I.pole_stride, B.s));
  }
  return HX_OK;
}

// defined with the step code below
void drop_graph(hx_plan* plan);
hx_status autotune(hx_plan* plan, char* ws, size_t ws_bytes, hipStream_t s);

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char* hx_status_str(int st) {
  switch (st) {
    case HX_OK: return "HX_OK";
    case HX_EINVAL: return "HX_EINVAL";
    case HX_ENOMEM: return "HX_ENOMEM";
    case HX_ESINGULAR: return "HX_ESINGULAR";
    case HX_EUNSTABLE: return "HX_EUNSTABLE";
    case HX_EDEVICE: return "HX_EDEVICE";
    case HX_ESTATE: return "HX_ESTATE";
    case HX_ESTAGE: return "HX_ESTAGE";
    default: return "HX_UNKNOWN";
  }
}

const char* hx_last_error(void) { return g_last_error.c_str(); }

hx_status hx_plan_create(hx_plan** out, int precision, int device, unsigned flags) {
  g_last_error.clear();
  if (!out) return fail(HX_EINVAL, "out is null");
  *out = nullptr;
  if (precision != HX_FP64 && precision != HX_FP32_REFINE)
    return fail(HX_EINVAL, "unsupported precision %d", precision);
  if (device < 0) return fail(HX_EINVAL, "device %d", device);
  if (flags & ~(HX_FLAG_ALLOW_UNSTABLE | HX_FLAG_NO_GRAPH | HX_FLAG_CHECK_STATE | HX_FLAG_UNBATCHED |
                HX_FLAG_AUTOTUNE | HX_FLAG_FUSED_MERGES))
    return fail(HX_EINVAL, "unknown flags 0x%x", flags);
  hx_plan* p = new hx_plan;
  p->device = device;
  p->precision = precision;
  p->flags = flags;
  *out = p;
  return HX_OK;
}

hx_status hx_plan_add(hx_plan* plan, const hx_mesh* mesh, const hx_coeffs* coeffs, double tau,
                      double delta, const hx_rational* rational, int nrhs, int* instance_id) {
  g_last_error.clear();
  if (!plan) return fail(HX_EINVAL, "plan is null");
  if (plan->arena) return fail(HX_ESTAGE, "plan is already bound");
  HX_TRY(validate_add(mesh, coeffs, tau, delta, rational, nrhs));
  Instance I;
  I.mesh = *mesh;
  I.q = mesh->p - 2;
  I.q2 = I.q * I.q;
  I.n_leaf = mesh->nex * mesh->ney;
  I.M = (rational->npoles - 1) / 2;
  I.npole = I.M + 1;
  I.nrhs = nrhs;
  I.ncol = I.npole * nrhs;
  I.tau = tau;
  I.delta = delta;
  I.fp32 = plan->precision == HX_FP32_REFINE;
  I.sw = coeffs->kind == HX_SW_SLIP;
  I.nfield = I.sw ? 3 : 2;
  if (I.sw) {
    I.f = coeffs->f;
    I.cw = std::sqrt(coeffs->gH);
    I.c2.assign((size_t)I.n_leaf * mesh->p * mesh->p, 1.0);   // Laplacian
    // interior-line operators on the q interior Chebyshev-Lobatto nodes
    const int q = I.q, N = mesh->p - 1;
    std::vector<double> x(q);
    for (int k = 0; k < q; ++k) x[k] = -std::cos((k + 1) * M_PI / N);
    std::vector<double> c(q, 1.0);
    for (int k = 0; k < q; ++k)
      for (int j = 0; j < q; ++j)
        if (j != k) c[k] *= x[k] - x[j];
    I.Dq.assign((size_t)q * q, 0.0);
    for (int i = 0; i < q; ++i) {
      double sum = 0.0;
      for (int j = 0; j < q; ++j)
        if (j != i) {
          I.Dq[i * q + j] = (c[i] / c[j]) / (x[i] - x[j]);
          sum += I.Dq[i * q + j];
        }
      I.Dq[i * q + i] = -sum;
    }
    I.w_lo.assign(q, 1.0);
    I.w_hi.assign(q, 1.0);
    for (int k = 0; k < q; ++k)
      for (int j = 0; j < q; ++j)
        if (j != k) {
          I.w_lo[k] *= (-1.0 - x[j]) / (x[k] - x[j]);
          I.w_hi[k] *= (1.0 - x[j]) / (x[k] - x[j]);
        }
  } else {
    I.c2.assign(coeffs->c2, coeffs->c2 + (size_t)I.n_leaf * mesh->p * mesh->p);
  }
  for (int k = 0; k < rational->npoles; ++k) {
    I.alpha.emplace_back(rational->alpha[2 * k], rational->alpha[2 * k + 1]);
    I.b.emplace_back(rational->b[2 * k], rational->b[2 * k + 1]);
  }
  check_fit(I);
  if (I.max_abs_R > 1.0 + 1e-6 && !(plan->flags & HX_FLAG_ALLOW_UNSTABLE))
    return fail(HX_EUNSTABLE, "max |R(ix)| = 1 + %.3g on the real line exceeds 1 + 1e-6",
                I.max_abs_R - 1.0);
  // pole table: folded poles m = 0..M
  cd beta = 0.0;
  for (auto& v : I.b) beta += v;
  I.beta = beta.real();
  auto d2 = [](cd z) { return make_double2(z.real(), z.imag()); };
  for (int k = 0; k <= I.M; ++k) {
    const cd a = I.alpha[I.M + k], bb = I.b[I.M + k];
    const double f = (k == 0) ? 1.0 : 2.0;
    PoleCoef pc;
    pc.alpha = d2(a);
    pc.cu = d2(f * bb);
    pc.cv = d2(f * bb * a);
    if (!I.sw) {   // g = (alpha u0 + tau v0) / tau^2
      pc.k1 = d2(a / (I.tau * I.tau));
      pc.k2 = d2(cd(1.0 / I.tau, 0.0));
      pc.k3 = d2(cd(0.0, 0.0));
      pc.sig = d2((a / I.tau) * (a / I.tau));
    } else {       // g = (s/(c^2 a)) eta0/tau + div/(c tau) - (f/(c a)) curl/tau
      const cd ap = a / I.tau, sp = ap * ap + I.f * I.f;
      const double c = I.cw;
      pc.k1 = d2(sp / (c * c * ap * I.tau));
      pc.k2 = d2(cd(1.0 / (c * I.tau), 0.0));
      pc.k3 = d2(-I.f / (c * ap * I.tau));
      pc.sig = d2(sp / (c * c));
      SwCoef sc;
      sc.c0 = d2(f * bb);
      sc.c1 = d2(f * bb * ap / sp);
      sc.c2 = d2(f * bb / sp);
      I.swcoef.push_back(sc);
    }
    I.coef.push_back(pc);
  }
  if (I.sw) {
    cd b1 = 0.0, b2 = 0.0;
    for (int k = 0; k < (int)I.alpha.size(); ++k) {
      const cd ap = I.alpha[k] / I.tau, sp = ap * ap + I.f * I.f;
      b1 += I.b[k] * ap / sp;
      b2 += I.b[k] / sp;
    }
    I.beta1 = b1.real();
    I.beta2 = b2.real();
  }
  const std::vector<double> D = cheb_diff(mesh->p);
  for (int k = 1; k <= I.q; ++k) I.nrow.push_back(D[0 * mesh->p + k]);
  for (int k = 1; k <= I.q; ++k) I.nrow.push_back(D[(mesh->p - 1) * mesh->p + k]);
  build_tree(I);
  for (auto& L : I.levels)
    if (L.max_x > 4096 || L.max_n3 > 4096)
      return fail(HX_EINVAL, "merge interface of %d nodes exceeds the 4096-node LDS limit", L.max_x);
  plan->inst.push_back(std::move(I));
  if (instance_id) *instance_id = (int)plan->inst.size() - 1;
  layout_arena(plan);
  return HX_OK;
}

hx_status hx_plan_query(const hx_plan* plan, hx_info* info) {
  g_last_error.clear();
  if (!plan || !info) return fail(HX_EINVAL, "null plan or info");
  if (plan->inst.empty()) return fail(HX_ESTAGE, "plan has no instance");
  hx_info r{};
  r.arena_bytes = plan->arena_bytes;
  r.max_abs_R = 0.0;
  r.fit_X = 1e300;
  size_t wmax = 0, wmin = 0;
  for (auto& I : plan->inst) {
    r.operator_bytes += I.cbytes() * (size_t)(I.leaf_ops + I.merge_ops) * I.npole;
    r.dof_state += (long long)I.nfield * I.n_leaf * I.q2 * I.nrhs;
    r.dof_nodes += (long long)I.nfield * I.n_leaf * I.mesh.p * I.mesh.p * I.nrhs;
    r.folded_poles += I.npole;
    // every stored entry is read once per column per step
    long long entries = 0;
    for (auto& L : I.leaves) entries += (long long)I.q2 * (I.q2 + L.e);
    for (size_t l = 1; l < I.levels.size(); ++l)
      for (auto& B : I.levels[l].boxes) {
        const long long ext = B.n1 + B.n2;
        entries += (long long)B.n3 * (ext + B.n3) + ext * B.n3;
      }
    entries += (long long)I.n_wall * I.n_wall;   // shallow water: root wall system
    // one sweep (FP64) or two (precision form) per step; batched right-hand
    // sides share each operator read
    const double sweeps = I.fp32 ? 2.0 : 1.0;
    const double reads = batched(plan, I) ? 1.0 : (double)I.nrhs;
    r.op_bytes_per_step += sweeps * (double)I.cbytes() * (double)entries * I.npole * reads;
    r.flops_per_step += sweeps * 8.0 * (double)entries * I.npole * I.nrhs;
    r.max_abs_R = std::max(r.max_abs_R, I.max_abs_R);
    r.fit_X = std::min(r.fit_X, I.fit_X);
    r.sum_abs_b = std::max(r.sum_abs_b, I.sum_abs_b);
    const size_t cap = (size_t)16 << 30;
    size_t all = ws_layout(I, I.npole).total;
    int ch = I.npole;
    while (all > cap && ch > 1) all = ws_layout(I, --ch).total;
    wmax = std::max(wmax, all);
    wmin = std::max(wmin, ws_layout(I, 1).total);
  }
  r.n_instances = (int)plan->inst.size();
  r.workspace_bytes = wmax;
  r.workspace_min_bytes = wmin;
  *info = r;
  return HX_OK;
}

hx_status hx_plan_bind(hx_plan* plan, void* arena, size_t arena_bytes) {
  g_last_error.clear();
  if (!plan || !arena) return fail(HX_EINVAL, "null plan or arena");
  if (plan->inst.empty()) return fail(HX_ESTAGE, "plan has no instance");
  if (plan->arena) return fail(HX_ESTAGE, "plan is already bound");
  if (reinterpret_cast<uintptr_t>(arena) % kAlign) return fail(HX_EINVAL, "arena not 256-byte aligned");
  if (arena_bytes < plan->arena_bytes)
    return fail(HX_ENOMEM, "arena of %zu bytes, %zu needed", arena_bytes, plan->arena_bytes);
  HIP_OK(hipSetDevice(plan->device));
  char* a = static_cast<char*>(arena);
  for (auto& I : plan->inst) {
    HIP_OK(hipMemcpy(a + I.d_leaves, I.leaves.data(), sizeof(LeafDesc) * I.leaves.size(), hipMemcpyHostToDevice));
    if (!I.idx.empty())
      HIP_OK(hipMemcpy(a + I.d_idx, I.idx.data(), sizeof(int) * I.idx.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(a + I.d_coef, I.coef.data(), sizeof(PoleCoef) * I.coef.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(a + I.d_nrow, I.nrow.data(), sizeof(double) * I.nrow.size(), hipMemcpyHostToDevice));
    if (I.sw || I.fp32) {
      const std::vector<double> D = cheb_diff(I.mesh.p);
      HIP_OK(hipMemcpy(a + I.d_D, D.data(), sizeof(double) * D.size(), hipMemcpyHostToDevice));
    }
    if (I.sw && I.fp32)
      HIP_OK(hipMemcpy(a + I.d_slotw, I.slot_wall.data(), sizeof(int) * I.slot_wall.size(), hipMemcpyHostToDevice));
    if (I.sw) {
      HIP_OK(hipMemcpy(a + I.d_wall, I.wall.data(), sizeof(int4) * I.wall.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(a + I.d_Dq, I.Dq.data(), sizeof(double) * I.Dq.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(a + I.d_wlo, I.w_lo.data(), sizeof(double) * I.w_lo.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(a + I.d_whi, I.w_hi.data(), sizeof(double) * I.w_hi.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(a + I.d_swc, I.swcoef.data(), sizeof(SwCoef) * I.swcoef.size(), hipMemcpyHostToDevice));
    }
    if (I.fp32)
      HIP_OK(hipMemcpy(a + I.d_c2, I.c2.data(), sizeof(double) * I.c2.size(), hipMemcpyHostToDevice));
    for (auto& L : I.levels)
      if (!L.boxes.empty())
        HIP_OK(hipMemcpy(a + L.d_boxes, L.boxes.data(), sizeof(BoxDesc) * L.boxes.size(), hipMemcpyHostToDevice));
  }
  plan->arena = a;
  plan->d_flag = reinterpret_cast<int*>(a + plan->d_flag_off);
  return HX_OK;
}

hx_status hx_plan_build(hx_plan* plan, void* workspace, size_t workspace_bytes, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(HX_EINVAL, "plan is null");
  if (!plan->arena) return fail(HX_ESTAGE, "plan is not bound");
  if (!workspace) return fail(HX_EINVAL, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(HX_EINVAL, "workspace not 256-byte aligned");
  HIP_OK(hipSetDevice(plan->device));
  Build B;
  B.plan = plan;
  B.s = static_cast<hipStream_t>(stream);
  B.ws = static_cast<char*>(workspace);
  B.ws_bytes = workspace_bytes;
  RB_OK(rocblas_create_handle(&B.rb));
  struct HandleGuard { rocblas_handle h; ~HandleGuard() { rocblas_destroy_handle(h); } } guard{B.rb};
  RB_OK(rocblas_set_stream(B.rb, B.s));
  plan->built = false;
  for (auto& I : plan->inst) {
    int ch = I.npole;
    while (ch > 0 && ws_layout(I, ch).total > workspace_bytes) --ch;
    if (ch == 0)
      return fail(HX_ENOMEM, "workspace of %zu bytes, at least %zu needed", workspace_bytes,
                  ws_layout(I, 1).total);
    const WsLayout W = ws_layout(I, ch);
    HX_TRY(upload(B, B.ws + W.c2, I.c2.data(), sizeof(double) * I.c2.size()));
    const std::vector<double> D = cheb_diff(I.mesh.p);
    HX_TRY(upload(B, B.ws + W.D, D.data(), sizeof(double) * D.size()));
    for (int p0 = 0; p0 < I.npole; p0 += ch) HX_TRY(build_chunk(B, I, W, p0, std::min(ch, I.npole - p0)));
  }
  HIP_OK(hipStreamSynchronize(B.s));
  drop_graph(plan);
  plan->tab_ready = false;
  if (plan->flags & HX_FLAG_FUSED_MERGES)
    for (Instance& I : plan->inst) I.tune_fuse[O_MERGE_UP] = I.tune_fuse[O_MERGE_DOWN] = 1;
  if (plan->flags & HX_FLAG_AUTOTUNE) HX_TRY(autotune(plan, B.ws, B.ws_bytes, B.s));
  plan->built = true;
  return HX_OK;
}

}  // extern "C"

namespace {

// Event pairs around kernel launches (diagnostic profiling of a step).
struct Prof {
  std::vector<hipEvent_t> start, stop;
  std::vector<int> cls;
  hipStream_t s = nullptr;
  hx_status begin(int c) {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    start.push_back(e);
    cls.push_back(c);
    HIP_OK(hipEventRecord(e, s));
    return HX_OK;
  }
  hx_status end() {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    stop.push_back(e);
    HIP_OK(hipEventRecord(e, s));
    return HX_OK;
  }
  ~Prof() {
    for (auto e : start) (void)hipEventDestroy(e);   // teardown: nothing to report
    for (auto e : stop) (void)hipEventDestroy(e);
  }
};

#define TIMED(cls, launch)                      \
  do {                                          \
    if (prof) HX_TRY(prof->begin(cls));         \
    HIP_OK(launch);                             \
    if (prof) HX_TRY(prof->end());              \
  } while (0)


// ---- batched instances: recorded stages, fused over instances ---------------------
//
// Every instance that runs on the matrix cores records its step as a list of
// stages (kernel kind, tile count, block count, LDS bytes and its argument
// block).  The stages of all instances are then ordered by (pass, stage,
// level) and stages of the same kind and tile count become ONE launch over
// the blocks of every instance in it, its arguments read from a table in the
// arena.  Levels are counted from the elements up, so an instance with fewer
// levels simply takes part in fewer merge launches; its own order (upward
// levels ascending, downward descending) is kept.

enum StageKind : int {
  K_LU_D, K_LU_F, K_MU_D, K_MU_F, K_MD_D, K_MD_F, K_LD_D, K_LD_F, K_LDS_D, K_LDS_F,
  K_ROOT_D, K_ROOT_F, K_RES_W, K_RES_S, K_PREP, K_WALL, K_POST_D, K_POST_F,
  K_MU2_D, K_MU2_F, K_MD2_D, K_MD2_F
};


struct Rec {
  int pass, order, level, kind, nt, wv, cls, inst;   // wv: merge waves / leaf staging variant
  long long blocks;
  size_t lds, args_size;
  unsigned char args[kArgsMax];
};

struct Recorder {
  std::vector<Rec> recs;
  template <class A>
  void add(int pass, int order, int level, int kind, int nt, long long blocks, size_t lds,
           const A& a, int cls, int inst, int wv = 4) {
    static_assert(sizeof(A) <= kArgsMax, "argument block too large");
    Rec r;
    r.pass = pass;
    r.order = order;
    r.level = level;
    r.kind = kind;
    r.nt = nt;
    r.wv = wv;
    r.cls = cls;
    r.inst = inst;
    r.blocks = blocks;
    r.lds = lds;
    r.args_size = sizeof(A);
    std::memcpy(r.args, &a, sizeof(A));
    recs.push_back(r);
  }
};

// Right-hand-side tile count of a stage: the tuned choice, else two tiles of
// 16 when there are more than 16 right-hand sides.
int stage_nt(const Instance& I, int order) {
  const int t = I.tune_nt[order];
  if (t == 1 || (t == 2 && I.nrhs > 16)) return t;
  return I.nrhs > 16 ? 2 : 1;
}

// Waves per block of a merge level with `rows` output rows: one wave (16
// rows per block) when the level's rows fit one 16-row tile, or when the
// tuned choice says so; four waves (64 rows per block) otherwise.
int merge_wv(const Instance& I, int order, int rows) {
  if (I.tune_wv[order] == 1) return 1;
  return rows <= 16 ? 1 : 4;
}

// Poles per block of an upward merge level whose launch would have `blocks` blocks
// with one pole each: as many as keep about kMergeBlocks blocks (one pole
// per block for levels with fewer), unless the tuner chose one pole per
// block.  A block then pays its descriptor and index loads once for the
// whole group.
constexpr long long kMergeBlocks = 4096;
int merge_pole_group(const Instance& I, int order, long long blocks) {
  if (I.tune_pg[order] == 1) return 1;
  return (int)std::max<long long>(1, std::min<long long>(I.npole, blocks / kMergeBlocks));
}

// When the tuner chose it, merge levels run in fused pairs (l, l + 1) from
// the elements up while a fused block's LDS stays within kFuseLds (two
// blocks or more per CU); by default every level has its own launch (the
// fused blocks hold so much LDS that few fit on a CU, and on the workloads
// measured the per-level launches were faster).  lds[l] > 0 marks the lower
// level l of a pair and holds the LDS bytes of its launch.
constexpr size_t kFuseLds = 64 * 1024;
template <class T>
std::vector<size_t> fused_pairs(const Instance& I, int order, int nt) {
  const size_t nl = I.levels.size();
  std::vector<size_t> lds(nl, 0);
  if (I.tune_fuse[order] != 1) return lds;
  auto r4 = [](int n) { return (n + 3) & ~3; };
  for (size_t l = 1; l + 1 < nl; l += 2) {
    size_t need = 0;
    for (const BoxDesc& Tb : I.levels[l + 1].boxes) {
      const BoxDesc& A = I.levels[l].boxes[Tb.a_box];
      const BoxDesc& B = I.levels[l].boxes[Tb.b_box];
      if (order == O_MERGE_UP) {
        const int child = A.n1 + A.n2 + B.n1 + B.n2 + 2 * (A.n3 + B.n3);
        const int mid = A.n1 + A.n2 + B.n1 + B.n2;
        const int stage = std::max(r4(A.n3) + r4(B.n3), r4(Tb.n3));
        need = std::max(need, hx::merge2_up_lds_bytes<T>(nt, child, mid, stage));
      } else {
        const int rows = r4(Tb.n1 + Tb.n2 + Tb.n3) + r4(A.n1 + A.n2 + A.n3) + r4(B.n1 + B.n2 + B.n3);
        need = std::max(need, hx::merge2_down_lds_bytes<T>(nt, rows));
      }
    }
    if (need > kFuseLds) break;   // the levels above are larger still
    lds[l] = need;
  }
  return lds;
}

// Tile count and source staging of the first upward element sweep: two
// tiles only while g fits in 64 KiB; the sources are staged (and a group of
// poles walked per block) while they fit beside g, unless the tuner chose
// otherwise.  The correction sweep never stages (its sources differ per pole).
struct LeafUpShape {
  int nt;
  bool staged;
};

template <class T>
LeafUpShape leaf_up_shape(const Instance& I) {
  const int nsrc = I.sw ? 3 : 2;
  int nt = stage_nt(I, O_LEAF_UP);
  if (nt == 2 && hx::leaf_up_lds_bytes<T>(I.q, 2, false, 0) > 65536) nt = 1;
  const bool staged = I.tune_xl != 2 && hx::leaf_up_lds_bytes<T>(I.q, nt, false, nsrc) <= 65536;
  return {nt, staged};
}

template <class T>
void record_instance(const hx_plan* plan, const Instance& I, int inst, double* state, Recorder& R) {
  using C = typename hx::Cplx<T>::type;
  constexpr bool refine = sizeof(T) == sizeof(float);
  constexpr bool dbl = !refine;
  char* a = plan->arena;
  const C* ops = reinterpret_cast<const C*>(a + I.d_ops);
  C* w = reinterpret_cast<C*>(a + I.d_w);
  const auto* leaves = reinterpret_cast<const LeafDesc*>(a + I.d_leaves);
  const auto* coef = reinterpret_cast<const PoleCoef*>(a + I.d_coef);
  const int* idx = reinterpret_cast<const int*>(a + I.d_idx);
  auto vec = [&](size_t off) { return reinterpret_cast<C*>(a + off); };
  auto dptr = [&](size_t off) { return reinterpret_cast<const double*>(a + off); };
  const bool sw = I.sw;
  const long long n_int = (long long)I.n_leaf * I.q2;
  const long long stride = (long long)I.nfield * n_int;
  const double sx = 2.0 * I.mesh.nex / (I.mesh.x1 - I.mesh.x0);
  const double sy = 2.0 * I.mesh.ney / (I.mesh.y1 - I.mesh.y0);
  double* prep = sw ? reinterpret_cast<double*>(a + I.d_prep) : nullptr;
  double* wallv = sw ? reinterpret_cast<double*>(a + I.d_wallv) : nullptr;
  const auto* wall = sw ? reinterpret_cast<const int4*>(a + I.d_wall) : nullptr;
  const auto* swc = sw ? reinterpret_cast<const SwCoef*>(a + I.d_swc) : nullptr;
  double2* dn = refine ? reinterpret_cast<double2*>(a + I.d_dn) : nullptr;
  C* gres = refine ? reinterpret_cast<C*>(a + I.d_gres) : nullptr;
  C* y0 = refine ? reinterpret_cast<C*>(a + I.d_y0) : nullptr;
  double* esum = (refine && sw) ? reinterpret_cast<double*>(a + I.d_esum) : nullptr;
  const double* src = sw ? prep : state;
  const size_t nl = I.levels.size();

  if (sw) {
    hx::SwPrepArgs pa{};
    pa.state = state;
    pa.prep = prep;
    pa.rhs_stride = stride;
    pa.n_int = (int)n_int;
    pa.nrhs = I.nrhs;
    pa.q = I.q;
    pa.Dq = dptr(I.d_Dq);
    pa.sx = sx;
    pa.sy = sy;
    R.add(0, O_PREP, 0, K_PREP, 1, (long long)I.n_leaf * I.nrhs, 0, pa, HX_K_SW_PREP, inst);
    hx::SwWallArgs wa{};
    wa.state = state;
    wa.rhs_stride = stride;
    wa.n_int = (int)n_int;
    wa.nrhs = I.nrhs;
    wa.q = I.q;
    wa.n_wall = I.n_wall;
    wa.wall = wall;
    wa.w_lo = dptr(I.d_wlo);
    wa.w_hi = dptr(I.d_whi);
    wa.out = wallv;
    R.add(0, O_PREP, 1, K_WALL, 1, ((long long)I.n_wall * I.nrhs + hx::kBlock - 1) / hx::kBlock, 0,
          wa, HX_K_SW_PREP, inst);
  }
  const int passes = refine ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    hx::MmLeafUpArgs<T> lu{};
    lu.ops = ops;
    lu.pole_stride = I.pole_stride;
    lu.leaves = leaves;
    lu.npole = I.npole;
    lu.nrhs = I.nrhs;
    lu.q = I.q;
    lu.state = src;
    lu.rhs_stride = sw ? 3 * n_int : stride;
    lu.n_int = (int)n_int;
    lu.nsrc = sw ? 3 : 2;
    lu.coef = coef;
    lu.inv_tau = 1.0 / I.tau;
    lu.inv_tau2 = 1.0 / (I.tau * I.tau);
    lu.nrow = dptr(I.d_nrow);
    lu.sx = sx;
    lu.sy = sy;
    lu.w = w;
    lu.w_pole = n_int;
    lu.h = vec(I.levels[0].d_h);
    lu.h_pole = I.levels[0].total_ext;
    lu.gin = pass ? gres : nullptr;
    // LDS: staged g, the w tile for h (when it fits), the staged source
    // fields (first sweep); two tiles only while g and the sources fit in
    // 64 KiB, and the w tile only while the total does
    // Staging the sources once per block and walking a group of poles pays
    // when the sources fit beside the staged g; otherwise one pole per block
    // reads them per pole (the tuner may also choose that on purpose).
    const LeafUpShape shape = leaf_up_shape<T>(I);
    const int nt = shape.nt;
    const bool xl = !pass && shape.staged;
    const int staged = xl ? lu.nsrc : 0;
    lu.x_lds = xl ? 1 : 0;
    lu.w_lds = hx::leaf_up_lds_bytes<T>(I.q, nt, true, staged) <= 65536 ? 1 : 0;
    const size_t lds = hx::leaf_up_lds_bytes<T>(I.q, nt, lu.w_lds != 0, staged);
    // poles per block when staging: all of them while elements x tiles give
    // >= 4096 blocks, else as many as keep ~4096 blocks
    const long long et = (long long)I.n_leaf * hx::mm_tiles(I.nrhs, nt);
    lu.pole_group = xl ? (int)std::max<long long>(1, std::min<long long>(I.npole, et * I.npole / 4096))
                       : 1;
    const long long npg = (I.npole + lu.pole_group - 1) / lu.pole_group;
    // (the group's variant field carries the staging choice: instances in
    // one fused launch share the kernel instantiation)
    R.add(pass, O_LEAF_UP, 0, dbl ? K_LU_D : K_LU_F, nt, et * npg, lds, lu, HX_K_LEAF_UP, inst,
          lu.x_lds);

    const int mu_nt = stage_nt(I, O_MERGE_UP);
    const std::vector<size_t> fu = fused_pairs<T>(I, O_MERGE_UP, mu_nt);
    for (size_t l = 1; l < nl; ++l) {
      if (fu[l]) {   // levels l and l + 1 in one launch
        hx::MmMerge2Args<T> m2{};
        m2.ops = ops;
        m2.pole_stride = I.pole_stride;
        m2.lo = reinterpret_cast<const BoxDesc*>(a + I.levels[l].d_boxes);
        m2.hi = reinterpret_cast<const BoxDesc*>(a + I.levels[l + 1].d_boxes);
        m2.idx = idx;
        m2.npole = I.npole;
        m2.nrhs = I.nrhs;
        m2.child = vec(I.levels[l - 1].d_h);
        m2.child_pole = I.levels[l - 1].total_ext;
        m2.self = vec(I.levels[l + 1].d_h);
        m2.self_pole = I.levels[l + 1].total_ext;
        m2.g3_lo = vec(I.levels[l].d_g3);
        m2.g3_lo_pole = I.levels[l].total_n3;
        m2.g3_hi = vec(I.levels[l + 1].d_g3);
        m2.g3_hi_pole = I.levels[l + 1].total_n3;
        m2.dn = pass ? dn : nullptr;
        m2.dn_pole = I.levels[0].total_ext;
        R.add(pass, O_MERGE_UP, (int)l, dbl ? K_MU2_D : K_MU2_F, mu_nt,
              (long long)I.levels[l + 1].boxes.size() * I.npole * hx::mm_tiles(I.nrhs, mu_nt), fu[l],
              m2, HX_K_MERGE_UP, inst, 0);
        ++l;
        continue;
      }
      const Level& L = I.levels[l];
      hx::MmMergeArgs<T> m{};
      m.ops = ops;
      m.pole_stride = I.pole_stride;
      m.boxes = reinterpret_cast<const BoxDesc*>(a + L.d_boxes);
      m.idx = idx;
      m.npole = I.npole;
      m.nrhs = I.nrhs;
      const int wv = merge_wv(I, O_MERGE_UP, L.max_ext);
      m.row_groups = std::max(1, (L.max_ext + 16 * wv - 1) / (16 * wv));
      m.child = vec(I.levels[l - 1].d_h);
      m.child_pole = I.levels[l - 1].total_ext;
      m.self = vec(L.d_h);
      m.self_pole = L.total_ext;
      m.g3 = vec(L.d_g3);
      m.g3_pole = L.total_n3;
      m.dn = pass ? dn : nullptr;
      m.dn_pole = I.levels[0].total_ext;
      const int mnt = stage_nt(I, O_MERGE_UP);
      const long long per_pole = (long long)L.boxes.size() * hx::mm_tiles(I.nrhs, mnt) * m.row_groups;
      m.pole_group = merge_pole_group(I, O_MERGE_UP, per_pole * I.npole);
      R.add(pass, O_MERGE_UP, (int)l, dbl ? K_MU_D : K_MU_F, mnt,
            per_pole * ((I.npole + m.pole_group - 1) / m.pole_group), 0, m, HX_K_MERGE_UP, inst, wv);
    }
    if (sw) {
      const Level& Rt = I.levels[nl - 1];
      hx::SwRootArgs<T> ra{};
      ra.ops = ops;
      ra.pole_stride = I.pole_stride;
      ra.q_off = I.q_off;
      ra.n = I.n_wall;
      ra.npole = I.npole;
      ra.nrhs = I.nrhs;
      ra.row_groups = (I.n_wall + 63) / 64;
      ra.coef = coef;
      ra.inv_tau = 1.0 / I.tau;
      ra.inv_c = 1.0 / I.cw;
      ra.f = I.f;
      ra.wall = wallv;
      ra.h = vec(Rt.d_h);
      ra.u = vec(Rt.d_u);
      ra.rw = pass ? dn : nullptr;
      ra.rw_pole = I.levels[0].total_ext;
      ra.wall_info = wall;
      const int rnt = stage_nt(I, O_ROOT);
      R.add(pass, O_ROOT, 0, dbl ? K_ROOT_D : K_ROOT_F, rnt,
            (long long)I.npole * hx::mm_tiles(I.nrhs, rnt) * ra.row_groups, 0, ra, HX_K_SW_ROOT, inst);
    }
    const int md_nt = stage_nt(I, O_MERGE_DOWN);
    const std::vector<size_t> fd = fused_pairs<T>(I, O_MERGE_DOWN, md_nt);
    for (size_t l = nl - 1; l >= 1; --l) {
      if (l >= 2 && fd[l - 1]) {   // levels l and l - 1 in one launch
        hx::MmMerge2Args<T> m2{};
        m2.ops = ops;
        m2.pole_stride = I.pole_stride;
        m2.lo = reinterpret_cast<const BoxDesc*>(a + I.levels[l - 1].d_boxes);
        m2.hi = reinterpret_cast<const BoxDesc*>(a + I.levels[l].d_boxes);
        m2.idx = idx;
        m2.npole = I.npole;
        m2.nrhs = I.nrhs;
        m2.child = vec(I.levels[l - 2].d_u);
        m2.child_pole = I.levels[l - 2].total_ext;
        m2.self = vec(I.levels[l].d_u);
        m2.self_pole = I.levels[l].total_ext;
        m2.g3_lo = vec(I.levels[l - 1].d_g3);
        m2.g3_lo_pole = I.levels[l - 1].total_n3;
        m2.g3_hi = vec(I.levels[l].d_g3);
        m2.g3_hi_pole = I.levels[l].total_n3;
        R.add(pass, O_MERGE_DOWN, -(int)l, dbl ? K_MD2_D : K_MD2_F, md_nt,
              (long long)I.levels[l].boxes.size() * I.npole * hx::mm_tiles(I.nrhs, md_nt), fd[l - 1],
              m2, HX_K_MERGE_DOWN, inst, 0);
        --l;
        continue;
      }
      const Level& L = I.levels[l];
      hx::MmMergeArgs<T> m{};
      m.ops = ops;
      m.pole_stride = I.pole_stride;
      m.boxes = reinterpret_cast<const BoxDesc*>(a + L.d_boxes);
      m.idx = idx;
      m.npole = I.npole;
      m.nrhs = I.nrhs;
      const int wv = merge_wv(I, O_MERGE_DOWN, L.max_n3);
      m.row_groups = std::max(1, (L.max_n3 + 16 * wv - 1) / (16 * wv));
      m.child = vec(I.levels[l - 1].d_u);
      m.child_pole = I.levels[l - 1].total_ext;
      m.self = vec(L.d_u);
      m.self_pole = L.total_ext;
      m.g3 = vec(L.d_g3);
      m.g3_pole = L.total_n3;
      const int mnt = stage_nt(I, O_MERGE_DOWN);
      m.pole_group = 1;   // one pole per block (the downward kernel has no pole loop)
      R.add(pass, O_MERGE_DOWN, -(int)l, dbl ? K_MD_D : K_MD_F, mnt,
            (long long)L.boxes.size() * I.npole * hx::mm_tiles(I.nrhs, mnt) * m.row_groups, 0, m,
            HX_K_MERGE_DOWN, inst, wv);
    }
    hx::MmLeafDownArgs<T> ld{};
    ld.ops = ops;
    ld.pole_stride = I.pole_stride;
    ld.leaves = leaves;
    ld.npole = I.npole;
    ld.nrhs = I.nrhs;
    ld.q = I.q;
    ld.row_groups = (I.q2 + 63) / 64;
    ld.u = vec(I.levels[0].d_u);
    ld.u_pole = I.levels[0].total_ext;
    ld.w = w;
    ld.w_pole = n_int;
    ld.coef = coef;
    ld.state = state;
    ld.rhs_stride = stride;
    ld.n_int = (int)n_int;
    ld.beta = I.beta;
    ld.inv_tau = 1.0 / I.tau;
    const int dnt = stage_nt(I, O_LEAF_DOWN);
    const long long tiles = hx::mm_tiles(I.nrhs, dnt);
    const bool fused_sum = !sw && pass == passes - 1;   // wave: pole sum fused into the last sweep
    if (fused_sum) {
      ld.y0 = refine ? y0 : nullptr;                    // precision form: y = y0 + w - S u_e
      R.add(pass, O_LEAF_DOWN, 0, dbl ? K_LDS_D : K_LDS_F, dnt,
            (long long)I.n_leaf * tiles * ld.row_groups, 0, ld, HX_K_LEAF_DOWN, inst);
    } else {
      ld.y0 = (refine && pass == 0) ? y0 : w;           // first sweep of the precision form: into y0
      R.add(pass, O_LEAF_DOWN, 0, dbl ? K_LD_D : K_LD_F, dnt,
            (long long)I.n_leaf * I.npole * tiles * ld.row_groups, 0, ld, HX_K_LEAF_DOWN, inst);
    }
    if (refine && pass == 0) {
      hx::ResidualArgs rs{};
      rs.leaves = leaves;
      rs.npole = I.npole;
      rs.nrhs = I.nrhs;
      rs.p = I.mesh.p;
      rs.q = I.q;
      rs.c2 = dptr(I.d_c2);
      rs.D = dptr(I.d_D);
      rs.sx = sx;
      rs.sy = sy;
      rs.tau = I.tau;
      rs.coef = coef;
      rs.state = src;
      rs.rhs_stride = sw ? 3 * n_int : stride;
      rs.n_int = (int)n_int;
      rs.y0 = reinterpret_cast<const float2*>(y0);
      rs.w_pole = n_int;
      rs.ue = reinterpret_cast<const float2*>(a + I.levels[0].d_u);
      rs.e_pole = I.levels[0].total_ext;
      rs.gres = reinterpret_cast<float2*>(gres);
      rs.dn = dn;
      rs.nsrc = sw ? 3 : 2;
      if (sw) {
        rs.n_leaf = I.n_leaf;
        rs.slot_wall = reinterpret_cast<const int*>(a + I.d_slotw);
        rs.wallv = wallv;
        rs.n_wall = I.n_wall;
        rs.Dq = dptr(I.d_Dq);
        rs.f = I.f;
        rs.inv_c = 1.0 / I.cw;
        rs.swc = swc;
        rs.esum = esum;
      }
      rs.RR = hx::residual_rr(rs);
      R.add(pass, O_RESIDUAL, 0, sw ? K_RES_S : K_RES_W, 1,
            (long long)I.n_leaf * ((I.nrhs + rs.RR - 1) / rs.RR),
            hx::residual_lds_bytes(rs.p, rs.RR, rs.nsrc), rs, HX_K_RESIDUAL, inst);
    }
  }
  if (sw) {
    hx::SwPostArgs<T> po{};
    po.leaves = leaves;
    po.npole = I.npole;
    po.nrhs = I.nrhs;
    po.p = I.mesh.p;
    po.q = I.q;
    po.D = dptr(I.d_D);
    po.coef = swc;
    po.y = w;
    po.y_pole = n_int;
    po.ue = vec(I.levels[0].d_u);
    po.e_pole = I.levels[0].total_ext;
    po.state = state;
    po.rhs_stride = stride;
    po.n_int = (int)n_int;
    po.sx = sx;
    po.sy = sy;
    po.c = I.cw;
    po.f = I.f;
    po.beta1 = I.beta1;
    po.beta2 = I.beta2;
    po.inv_tau = 1.0 / I.tau;
    po.esum = esum;
    po.n_leaf = I.n_leaf;
    po.RR = hx::sw_post_rr(po.p, po.nrhs);
    R.add(passes - 1, O_POST, 0, dbl ? K_POST_D : K_POST_F, 1,
          (long long)I.n_leaf * ((I.nrhs + po.RR - 1) / po.RR), hx::sw_post_lds_bytes(po.p, po.RR),
          po, HX_K_POLE_SUM, inst);
  }
}

// Record every batched instance (states may be null for a count).
void record_all(const hx_plan* plan, double* const* states, Recorder& R) {
  for (size_t k = 0; k < plan->inst.size(); ++k) {
    const Instance& I = plan->inst[k];
    if (!batched(plan, I)) continue;
    double* st = states ? states[k] : nullptr;
    if (I.fp32) record_instance<float>(plan, I, (int)k, st, R);
    else record_instance<double>(plan, I, (int)k, st, R);
  }
}

// Order the stages, form the groups and pack their tables (argument
// blocks, then n + 1 block offsets) at 256-byte aligned offsets.
void group_stages(Recorder& R, std::vector<Group>& groups, std::vector<unsigned char>& blob) {
  std::stable_sort(R.recs.begin(), R.recs.end(), [](const Rec& x, const Rec& y) {
    if (x.pass != y.pass) return x.pass < y.pass;
    if (x.order != y.order) return x.order < y.order;
    if (x.level != y.level) return x.level < y.level;
    if (x.kind != y.kind) return x.kind < y.kind;
    if (x.nt != y.nt) return x.nt < y.nt;
    return x.wv < y.wv;
  });
  groups.clear();
  blob.clear();
  size_t i = 0;
  while (i < R.recs.size()) {
    size_t j = i;
    const Rec& h = R.recs[i];
    while (j < R.recs.size() && R.recs[j].pass == h.pass && R.recs[j].order == h.order &&
           R.recs[j].level == h.level && R.recs[j].kind == h.kind && R.recs[j].nt == h.nt &&
           R.recs[j].wv == h.wv)
      ++j;
    Group g{};
    g.kind = h.kind;
    g.nt = h.nt;
    g.wv = h.wv;
    g.cls = h.cls;
    g.n = (int)(j - i);
    g.args_off = align_up(blob.size());
    blob.resize(g.args_off + h.args_size * g.n);
    std::vector<int> first(g.n + 1, 0);
    long long b = 0;
    for (size_t k = i; k < j; ++k) {
      std::memcpy(blob.data() + g.args_off + (k - i) * h.args_size, R.recs[k].args, h.args_size);
      first[k - i] = (int)b;
      b += R.recs[k].blocks;
      g.lds = std::max(g.lds, R.recs[k].lds);
    }
    first[g.n] = (int)b;
    g.blocks = b;
    g.first_off = align_up(blob.size());
    blob.resize(g.first_off + sizeof(int) * first.size());
    std::memcpy(blob.data() + g.first_off, first.data(), sizeof(int) * first.size());
    groups.push_back(g);
    i = j;
  }
  blob.resize(align_up(blob.size()));
}

template <class A>
hx::Multi<A> multi_of(const hx_plan* plan, const Group& g) {
  hx::Multi<A> m;
  m.args = reinterpret_cast<const A*>(plan->arena + plan->d_tab + g.args_off);
  m.first = reinterpret_cast<const int*>(plan->arena + plan->d_tab + g.first_off);
  m.n = g.n;
  return m;
}

template <class A>
const A& host_args(const unsigned char* blob, const Group& g) {
  return *reinterpret_cast<const A*>(blob + g.args_off);
}

// A group of one instance: the single-instance kernel, arguments by value.
hipError_t launch_one(const unsigned char* blob, const Group& g, hipStream_t s) {
  const int b = (int)g.blocks;
  switch (g.kind) {
    case K_LU_D: return hx::launch_leaf_up_mm_one<double>(host_args<hx::MmLeafUpArgs<double>>(blob, g), b, g.nt, g.lds, s);
    case K_LU_F: return hx::launch_leaf_up_mm_one<float>(host_args<hx::MmLeafUpArgs<float>>(blob, g), b, g.nt, g.lds, s);
    case K_MU_D: return hx::launch_merge_up_mm_one<double>(host_args<hx::MmMergeArgs<double>>(blob, g), b, g.nt, g.wv, s);
    case K_MU_F: return hx::launch_merge_up_mm_one<float>(host_args<hx::MmMergeArgs<float>>(blob, g), b, g.nt, g.wv, s);
    case K_MD_D: return hx::launch_merge_down_mm_one<double>(host_args<hx::MmMergeArgs<double>>(blob, g), b, g.nt, g.wv, s);
    case K_MD_F: return hx::launch_merge_down_mm_one<float>(host_args<hx::MmMergeArgs<float>>(blob, g), b, g.nt, g.wv, s);
    case K_LD_D: return hx::launch_leaf_down_mm_one<double>(host_args<hx::MmLeafDownArgs<double>>(blob, g), b, g.nt, s);
    case K_LD_F: return hx::launch_leaf_down_mm_one<float>(host_args<hx::MmLeafDownArgs<float>>(blob, g), b, g.nt, s);
    case K_LDS_D: return hx::launch_leaf_down_sum_mm_one<double>(host_args<hx::MmLeafDownArgs<double>>(blob, g), b, g.nt, s);
    case K_LDS_F: return hx::launch_leaf_down_sum_mm_one<float>(host_args<hx::MmLeafDownArgs<float>>(blob, g), b, g.nt, s);
    case K_ROOT_D: return hx::launch_sw_root_mm_one<double>(host_args<hx::SwRootArgs<double>>(blob, g), b, g.nt, s);
    case K_ROOT_F: return hx::launch_sw_root_mm_one<float>(host_args<hx::SwRootArgs<float>>(blob, g), b, g.nt, s);
    case K_RES_W: return hx::launch_residual_one(host_args<hx::ResidualArgs>(blob, g), b, false, g.lds, s);
    case K_RES_S: return hx::launch_residual_one(host_args<hx::ResidualArgs>(blob, g), b, true, g.lds, s);
    case K_PREP: return hx::launch_sw_prep_one(host_args<hx::SwPrepArgs>(blob, g), b, s);
    case K_WALL: return hx::launch_sw_wall_one(host_args<hx::SwWallArgs>(blob, g), b, s);
    case K_POST_D: return hx::launch_sw_post_one<double>(host_args<hx::SwPostArgs<double>>(blob, g), b, g.lds, s);
    case K_POST_F: return hx::launch_sw_post_one<float>(host_args<hx::SwPostArgs<float>>(blob, g), b, g.lds, s);
    case K_MU2_D: return hx::launch_merge2_up_mm_one<double>(host_args<hx::MmMerge2Args<double>>(blob, g), b, g.nt, g.lds, s);
    case K_MU2_F: return hx::launch_merge2_up_mm_one<float>(host_args<hx::MmMerge2Args<float>>(blob, g), b, g.nt, g.lds, s);
    case K_MD2_D: return hx::launch_merge2_down_mm_one<double>(host_args<hx::MmMerge2Args<double>>(blob, g), b, g.nt, g.lds, s);
    case K_MD2_F: return hx::launch_merge2_down_mm_one<float>(host_args<hx::MmMerge2Args<float>>(blob, g), b, g.nt, g.lds, s);
  }
  return hipErrorInvalidValue;
}

// blob: the host copy of the tables the group was packed into.
hipError_t launch_group(const hx_plan* plan, const Group& g, const unsigned char* blob, hipStream_t s) {
  if (g.n == 1) return launch_one(blob, g, s);
  const int b = (int)g.blocks;
  switch (g.kind) {
    case K_LU_D: return hx::launch_leaf_up_mm_multi<double>(multi_of<hx::MmLeafUpArgs<double>>(plan, g), b, g.nt, g.wv != 0, g.lds, s);
    case K_LU_F: return hx::launch_leaf_up_mm_multi<float>(multi_of<hx::MmLeafUpArgs<float>>(plan, g), b, g.nt, g.wv != 0, g.lds, s);
    case K_MU_D: return hx::launch_merge_up_mm_multi<double>(multi_of<hx::MmMergeArgs<double>>(plan, g), b, g.nt, g.wv, s);
    case K_MU_F: return hx::launch_merge_up_mm_multi<float>(multi_of<hx::MmMergeArgs<float>>(plan, g), b, g.nt, g.wv, s);
    case K_MD_D: return hx::launch_merge_down_mm_multi<double>(multi_of<hx::MmMergeArgs<double>>(plan, g), b, g.nt, g.wv, s);
    case K_MD_F: return hx::launch_merge_down_mm_multi<float>(multi_of<hx::MmMergeArgs<float>>(plan, g), b, g.nt, g.wv, s);
    case K_LD_D: return hx::launch_leaf_down_mm_multi<double>(multi_of<hx::MmLeafDownArgs<double>>(plan, g), b, g.nt, s);
    case K_LD_F: return hx::launch_leaf_down_mm_multi<float>(multi_of<hx::MmLeafDownArgs<float>>(plan, g), b, g.nt, s);
    case K_LDS_D: return hx::launch_leaf_down_sum_mm_multi<double>(multi_of<hx::MmLeafDownArgs<double>>(plan, g), b, g.nt, s);
    case K_LDS_F: return hx::launch_leaf_down_sum_mm_multi<float>(multi_of<hx::MmLeafDownArgs<float>>(plan, g), b, g.nt, s);
    case K_ROOT_D: return hx::launch_sw_root_mm_multi<double>(multi_of<hx::SwRootArgs<double>>(plan, g), b, g.nt, s);
    case K_ROOT_F: return hx::launch_sw_root_mm_multi<float>(multi_of<hx::SwRootArgs<float>>(plan, g), b, g.nt, s);
    case K_RES_W: return hx::launch_residual_multi(multi_of<hx::ResidualArgs>(plan, g), b, false, g.lds, s);
    case K_RES_S: return hx::launch_residual_multi(multi_of<hx::ResidualArgs>(plan, g), b, true, g.lds, s);
    case K_PREP: return hx::launch_sw_prep_multi(multi_of<hx::SwPrepArgs>(plan, g), b, s);
    case K_WALL: return hx::launch_sw_wall_multi(multi_of<hx::SwWallArgs>(plan, g), b, s);
    case K_POST_D: return hx::launch_sw_post_multi<double>(multi_of<hx::SwPostArgs<double>>(plan, g), b, g.lds, s);
    case K_POST_F: return hx::launch_sw_post_multi<float>(multi_of<hx::SwPostArgs<float>>(plan, g), b, g.lds, s);
    case K_MU2_D: return hx::launch_merge2_up_mm_multi<double>(multi_of<hx::MmMerge2Args<double>>(plan, g), b, g.nt, g.lds, s);
    case K_MU2_F: return hx::launch_merge2_up_mm_multi<float>(multi_of<hx::MmMerge2Args<float>>(plan, g), b, g.nt, g.lds, s);
    case K_MD2_D: return hx::launch_merge2_down_mm_multi<double>(multi_of<hx::MmMerge2Args<double>>(plan, g), b, g.nt, g.lds, s);
    case K_MD2_F: return hx::launch_merge2_down_mm_multi<float>(multi_of<hx::MmMerge2Args<float>>(plan, g), b, g.nt, g.lds, s);
  }
  return hipErrorInvalidValue;
}

// Record the batched instances for these states, group their stages and
// upload the tables (stream-ordered, then waited for: never inside a
// capture).  Skipped when the tables already match the states.
hx_status prepare_tables(hx_plan* plan, double* const* states, hipStream_t s) {
  std::vector<double*> key(states, states + plan->inst.size());
  if (plan->tab_ready && key == plan->tab_states) return HX_OK;
  Recorder R;
  record_all(plan, states, R);
  group_stages(R, plan->groups, plan->tab_blob);
  if (plan->tab_blob.size() > plan->tab_bytes)
    return fail(HX_ENOMEM, "stage tables of %zu bytes exceed the %zu reserved", plan->tab_blob.size(),
                plan->tab_bytes);
  for (const Group& g : plan->groups)
    if (g.blocks > 0x7fffffffLL) return fail(HX_EINVAL, "a fused launch exceeds 2^31 blocks");
  if (!plan->tab_blob.empty()) {
    HIP_OK(hipMemcpyAsync(plan->arena + plan->d_tab, plan->tab_blob.data(), plan->tab_blob.size(),
                          hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  plan->tab_states = key;
  plan->tab_ready = true;
  return HX_OK;
}

// Stages the tile count is tuned for (stage order of the recorder), in the
// order of the HX_STAGE_* codes.
constexpr int kTunedOrders[HX_STAGES] = {O_LEAF_UP, O_MERGE_UP, O_ROOT, O_MERGE_DOWN, O_LEAF_DOWN};

// Autotuner: for every batched instance and every tuned stage, launch that
// stage of every sweep (all its levels) in each candidate shape on a
// scratch state in the build workspace, time the best of five runs of
// each, keep the fastest.  Candidates: 1 or 2 right-hand-side tiles per
// block (more than 16 right-hand sides only); for the merge stages also
// one-wave blocks at every level against the level rule of merge_wv, and
// one pole per block against the pole groups of merge_pole_group; for the
// upward element sweep, staged sources against none.
template <class T>
hx_status tune_instance(hx_plan* plan, Instance& I, int k, double* scratch, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1) {
  for (int st = 0; st < HX_STAGES; ++st) {
    const int order = kTunedOrders[st];
    const bool merge = order == O_MERGE_UP || order == O_MERGE_DOWN;
    const bool up = order == O_LEAF_UP;
    // (tiles, shape mode): merges bit 0 = one-wave blocks (else the level
    // rule), upward merges bit 1 = one pole per block (else pole groups),
    // merges bit 2 = fused pairs of low levels (else one launch per level);
    // upward elements 0 = stage the sources when they fit / 2 = never
    std::vector<std::pair<int, int>> cand;
    for (int nt = 1; nt <= (I.nrhs > 16 ? 2 : 1); ++nt)
      for (int v : (order == O_MERGE_UP     ? std::vector<int>{0, 1, 2, 3, 4, 5, 6, 7}
                    : order == O_MERGE_DOWN ? std::vector<int>{0, 1, 4, 5}
                    : up                    ? std::vector<int>{0, 2}
                                            : std::vector<int>{0}))
        cand.push_back({nt, v});
    if (cand.size() < 2) continue;
    // the default shape first; another shape replaces the best so far only
    // when at least 1% faster, so that timing noise does not flip choices
    const std::pair<int, int> dflt{I.nrhs > 16 ? 2 : 1, 0};
    std::stable_partition(cand.begin(), cand.end(), [&](const std::pair<int, int>& c) { return c == dflt; });
    float best = 1e30f;
    std::pair<int, int> best_c{0, 0};
    for (const auto& c : cand) {
      I.tune_nt[order] = I.nrhs > 16 ? c.first : 0;
      if (merge) {
        I.tune_wv[order] = c.second & 1;
        I.tune_pg[order] = (c.second >> 1) & 1;
        I.tune_fuse[order] = (c.second >> 2) & 1;
      }
      if (up) I.tune_xl = c.second;
      Recorder R;
      record_instance<T>(plan, I, k, scratch, R);
      Recorder one;
      // the stage in every sweep of the step (the precision form's
      // correction sweep runs other kernels for some stages, e.g. the
      // downward elements fused with the pole sum)
      for (const Rec& r : R.recs)
        if (r.order == order) one.recs.push_back(r);
      if (one.recs.empty()) break;
      std::vector<Group> groups;
      std::vector<unsigned char> blob;
      group_stages(one, groups, blob);
      if (blob.size() > plan->tab_bytes) break;
      HIP_OK(hipMemcpyAsync(plan->arena + plan->d_tab, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
      HIP_OK(hipStreamSynchronize(s));
      float t_min = 1e30f;
      for (int rep = 0; rep < 6; ++rep) {   // the first run warms up
        HIP_OK(hipEventRecord(e0, s));
        for (const Group& g : groups) HIP_OK(launch_group(plan, g, blob.data(), s));
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) t_min = std::min(t_min, ms);
      }
      if (t_min < best * 0.99f) {
        best = t_min;
        best_c = c;
      }
    }
    I.tune_nt[order] = I.nrhs > 16 ? best_c.first : 0;
    if (merge) {
      I.tune_wv[order] = best_c.second & 1;
      I.tune_pg[order] = (best_c.second >> 1) & 1;
      I.tune_fuse[order] = (best_c.second >> 2) & 1;
    }
    if (up) I.tune_xl = best_c.second;
  }
  return HX_OK;
}

hx_status autotune(hx_plan* plan, char* ws, size_t ws_bytes, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } g{e0, e1};
  hx_status st = HX_OK;
  for (size_t k = 0; k < plan->inst.size() && st == HX_OK; ++k) {
    Instance& I = plan->inst[k];
    if (!batched(plan, I)) continue;
    const size_t need = sizeof(double) * (size_t)I.nfield * I.n_leaf * I.q2 * I.nrhs;
    if (need > ws_bytes) continue;                 // no room for a scratch state: default rule
    double* scratch = reinterpret_cast<double*>(ws);
    HIP_OK(hipMemsetAsync(scratch, 0, need, s));
    st = I.fp32 ? tune_instance<float>(plan, I, (int)k, scratch, s, e0, e1)
                : tune_instance<double>(plan, I, (int)k, scratch, s, e0, e1);
  }
  plan->tab_ready = false;                         // the tables now hold tuning stages
  return st;
}

hx_status enqueue_single(hx_plan* plan, const Instance& I, double* state, hipStream_t s, Prof* prof) {
  char* a = plan->arena;
  const double2* ops = reinterpret_cast<const double2*>(a + I.d_ops);
  double2* w = reinterpret_cast<double2*>(a + I.d_w);
  const auto* leaves = reinterpret_cast<const LeafDesc*>(a + I.d_leaves);
  const auto* coef = reinterpret_cast<const PoleCoef*>(a + I.d_coef);
  const int* idx = reinterpret_cast<const int*>(a + I.d_idx);
  const long long n_int = (long long)I.n_leaf * I.q2;
  auto vec = [&](size_t off) { return reinterpret_cast<double2*>(a + off); };

  hx::LeafUpArgs lu{};
  lu.ops = ops;
  lu.pole_stride = I.pole_stride;
  lu.leaves = leaves;
  lu.ncol = I.ncol;
  lu.nrhs = I.nrhs;
  lu.state = state;
  lu.rhs_stride = 2 * n_int;
  lu.n_int = (int)n_int;
  lu.nsrc = 2;
  lu.coef = coef;
  lu.inv_tau = 1.0 / I.tau;
  lu.inv_tau2 = 1.0 / (I.tau * I.tau);
  lu.nrow = reinterpret_cast<const double*>(a + I.d_nrow);
  lu.sx = 2.0 * I.mesh.nex / (I.mesh.x1 - I.mesh.x0);
  lu.sy = 2.0 * I.mesh.ney / (I.mesh.y1 - I.mesh.y0);
  lu.q = I.q;
  lu.w = w;
  lu.w_pole = n_int;
  lu.h = vec(I.levels[0].d_h);
  lu.h_pole = I.levels[0].total_ext;
  TIMED(HX_K_LEAF_UP, hx::launch_leaf_up(lu, I.n_leaf, s));

  const size_t nl = I.levels.size();
  for (size_t l = 1; l < nl; ++l) {
    const Level& L = I.levels[l];
    hx::MergeArgs m{};
    m.ops = ops;
    m.pole_stride = I.pole_stride;
    m.boxes = reinterpret_cast<const BoxDesc*>(a + L.d_boxes);
    m.idx = idx;
    m.ncol = I.ncol;
    m.nrhs = I.nrhs;
    m.row_blocks = std::max(1, (L.max_ext + hx::kBlock - 1) / hx::kBlock);
    m.child = vec(I.levels[l - 1].d_h);
    m.child_pole = I.levels[l - 1].total_ext;
    m.self = vec(L.d_h);
    m.self_pole = L.total_ext;
    m.g3 = vec(L.d_g3);
    m.g3_pole = L.total_n3;
    TIMED(HX_K_MERGE_UP, hx::launch_merge_up(m, (int)L.boxes.size(), L.max_n3, s));
  }
  for (size_t l = nl - 1; l >= 1; --l) {
    const Level& L = I.levels[l];
    hx::MergeArgs m{};
    m.ops = ops;
    m.pole_stride = I.pole_stride;
    m.boxes = reinterpret_cast<const BoxDesc*>(a + L.d_boxes);
    m.idx = idx;
    m.ncol = I.ncol;
    m.nrhs = I.nrhs;
    m.row_blocks = std::max(1, (L.max_n3 + hx::kBlock - 1) / hx::kBlock);
    m.child = vec(I.levels[l - 1].d_u);
    m.child_pole = I.levels[l - 1].total_ext;
    m.self = vec(L.d_u);
    m.self_pole = L.total_ext;
    m.g3 = vec(L.d_g3);
    m.g3_pole = L.total_n3;
    TIMED(HX_K_MERGE_DOWN, hx::launch_merge_down(m, (int)L.boxes.size(), L.max_x, s));
  }
  hx::LeafDownArgs ld{};
  ld.ops = ops;
  ld.pole_stride = I.pole_stride;
  ld.leaves = leaves;
  ld.ncol = I.ncol;
  ld.nrhs = I.nrhs;
  ld.q = I.q;
  ld.u = vec(I.levels[0].d_u);
  ld.u_pole = I.levels[0].total_ext;
  ld.w = w;
  ld.w_pole = n_int;
  TIMED(HX_K_LEAF_DOWN, hx::launch_leaf_down(ld, I.n_leaf, s));
  return HX_OK;
}

// One step of every instance.  The stage tables of the batched instances
// must have been prepared for these states (prepare_tables).
hx_status enqueue_step(hx_plan* plan, double* const* states, hipStream_t s, Prof* prof = nullptr) {
  char* a = plan->arena;
  for (size_t k = 0; k < plan->inst.size(); ++k) {
    Instance& I = plan->inst[k];
    if (batched(plan, I)) continue;
    HX_TRY(enqueue_single(plan, I, states[k], s, prof));
    const long long n_int = (long long)I.n_leaf * I.q2;
    hx::PoleSumArgs ps{};
    ps.leaves = reinterpret_cast<const LeafDesc*>(a + I.d_leaves);
    ps.npole = I.npole;
    ps.nrhs = I.nrhs;
    ps.q = I.q;
    ps.coef = reinterpret_cast<const PoleCoef*>(a + I.d_coef);
    ps.y = reinterpret_cast<const double2*>(a + I.d_w);
    ps.y_pole = n_int;
    ps.state = states[k];
    ps.rhs_stride = 2 * n_int;
    ps.n_int = (int)n_int;
    ps.beta = I.beta;
    ps.inv_tau = 1.0 / I.tau;
    TIMED(HX_K_POLE_SUM, hx::launch_pole_sum(ps, I.n_leaf, s));
  }
  for (const Group& g : plan->groups) TIMED(g.cls, launch_group(plan, g, plan->tab_blob.data(), s));
  return HX_OK;
}

void drop_graph(hx_plan* plan) {
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  plan->graph_exec = nullptr;
  plan->graph = nullptr;
  plan->graph_states.clear();
}

}  // namespace

extern "C" {

hx_status hx_step(hx_plan* plan, double* const* states, int n_steps, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(HX_EINVAL, "plan is null");
  if (!plan->built) return fail(HX_ESTAGE, "plan is not built");
  if (!states) return fail(HX_EINVAL, "states is null");
  if (n_steps < 0) return fail(HX_EINVAL, "n_steps = %d", n_steps);
  for (size_t k = 0; k < plan->inst.size(); ++k)
    if (!states[k]) return fail(HX_EINVAL, "state pointer %zu is null", k);
  if (n_steps == 0) return HX_OK;
  HIP_OK(hipSetDevice(plan->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->flags & HX_FLAG_CHECK_STATE) {
    HIP_OK(hipMemsetAsync(plan->d_flag, 0, sizeof(int), s));
    for (size_t k = 0; k < plan->inst.size(); ++k) {
      const Instance& I = plan->inst[k];
      HIP_OK(hx::launch_nonfinite_check(states[k], (long long)I.nfield * I.n_leaf * I.q2 * I.nrhs, plan->d_flag, s));
    }
    int flag = 0;
    HIP_OK(hipMemcpyAsync(&flag, plan->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (flag) return fail(HX_ESTATE, "non-finite value in the state");
  }
  HX_TRY(prepare_tables(plan, states, s));
  const bool use_graph = !(plan->flags & HX_FLAG_NO_GRAPH) && s != nullptr;
  if (!use_graph) {
    for (int n = 0; n < n_steps; ++n) HX_TRY(enqueue_step(plan, states, s));
    return HX_OK;
  }
  std::vector<double*> key(states, states + plan->inst.size());
  if (!plan->graph_exec || key != plan->graph_states) {
    drop_graph(plan);
    HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hx_status st = enqueue_step(plan, states, s);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (st != HX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    HIP_OK(ec);
    plan->graph = g;
    HIP_OK(hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0));
    plan->graph_states = key;
  }
  for (int n = 0; n < n_steps; ++n) HIP_OK(hipGraphLaunch(plan->graph_exec, s));
  return HX_OK;
}

hx_status hx_step_profile(hx_plan* plan, double* const* states, int n_steps, void* stream,
                          double* kernel_ms, int* launches, int n_classes) {
  g_last_error.clear();
  if (!plan) return fail(HX_EINVAL, "plan is null");
  if (!plan->built) return fail(HX_ESTAGE, "plan is not built");
  if (!states || !kernel_ms || !launches) return fail(HX_EINVAL, "null argument");
  if (n_steps < 0 || n_classes < 0) return fail(HX_EINVAL, "negative count");
  for (size_t k = 0; k < plan->inst.size(); ++k)
    if (!states[k]) return fail(HX_EINVAL, "state pointer %zu is null", k);
  for (int c = 0; c < n_classes; ++c) { kernel_ms[c] = 0.0; launches[c] = 0; }
  HIP_OK(hipSetDevice(plan->device));
  Prof prof;
  prof.s = static_cast<hipStream_t>(stream);
  HX_TRY(prepare_tables(plan, states, prof.s));
  for (int n = 0; n < n_steps; ++n) HX_TRY(enqueue_step(plan, states, prof.s, &prof));
  HIP_OK(hipStreamSynchronize(prof.s));
  for (size_t k = 0; k < prof.cls.size(); ++k) {
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, prof.start[k], prof.stop[k]));
    const int c = prof.cls[k];
    if (c < n_classes) {
      kernel_ms[c] += ms;
      launches[c] += 1;
    }
  }
  return HX_OK;
}

hx_status hx_plan_tiles(const hx_plan* plan, int instance, int* tiles, int n) {
  g_last_error.clear();
  if (!plan || !tiles) return fail(HX_EINVAL, "null plan or tiles");
  if (instance < 0 || instance >= (int)plan->inst.size())
    return fail(HX_EINVAL, "instance %d of %zu", instance, plan->inst.size());
  const Instance& I = plan->inst[instance];
  for (int st = 0; st < std::min(n, (int)HX_STAGES); ++st)
    tiles[st] = batched(plan, I) ? stage_nt(I, kTunedOrders[st]) : 0;
  return HX_OK;
}

hx_status hx_plan_variants(const hx_plan* plan, int instance, int* variants, int n) {
  g_last_error.clear();
  if (!plan || !variants) return fail(HX_EINVAL, "null plan or variants");
  if (instance < 0 || instance >= (int)plan->inst.size())
    return fail(HX_EINVAL, "instance %d of %zu", instance, plan->inst.size());
  const Instance& I = plan->inst[instance];
  const bool b = batched(plan, I);
  const bool f32 = I.fp32;
  for (int st = 0; st < std::min(n, (int)HX_STAGES); ++st) {
    const int order = kTunedOrders[st];
    int v = 0;
    if (b && st == HX_STAGE_LEAF_UP)
      v = (f32 ? leaf_up_shape<float>(I) : leaf_up_shape<double>(I)).staged ? 1 : 0;
    else if (b && (st == HX_STAGE_MERGE_UP || st == HX_STAGE_MERGE_DOWN)) {
      // fused pairs count only where some pair fits the LDS bound
      const int nt = stage_nt(I, order);
      const std::vector<size_t> fp = f32 ? fused_pairs<float>(I, order, nt) : fused_pairs<double>(I, order, nt);
      const bool fused = std::any_of(fp.begin(), fp.end(), [](size_t x) { return x > 0; });
      v = (I.tune_wv[order] == 1 ? 1 : 0) | (I.tune_pg[order] == 1 ? 2 : 0) | (fused ? 4 : 0);
    }
    variants[st] = v;
  }
  return HX_OK;
}

void hx_plan_destroy(hx_plan* plan) {
  if (!plan) return;
  drop_graph(plan);
  delete plan;
}

}  // extern "C"
