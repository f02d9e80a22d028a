/*
 * hpsexp — rational-approximation time stepping on MI355X (gfx950).
 *
 * Applies one large time step of a linear wave problem u_t = L u,
 *     exp(tau L) u  ~  R(tau L) u = sum_{m=-M}^{M} b_m (tau L - alpha_m)^{-1} u,
 * n times in a row (Haut, Babb, Martinsson, Wingate, arXiv:1402.5168,
 * section 1.2, eq. def_RM and the error bound eq. error-in-exp(t*L)).
 * Each resolvent is reduced to a complex-shifted elliptic solve (section
 * 2.1) on a multidomain Chebyshev collocation mesh (section 2.2), done by
 * the solve stage of a precomputed hierarchical direct solver (section
 * 2.3): dense per-element solution operators, then an upward and a
 * downward sweep over a binary merge tree of interface operators.
 *
 * Problems handled: linearised rotating shallow water with slip walls
 * (HX_SW_SLIP, below) and the wave equation in first-order form
 *     u_t = v,   v_t = div(c(x)^2 grad u)   on a rectangle,
 * with homogeneous Dirichlet data (HX_WAVE_DIRICHLET), for which
 *     (tau L - alpha)(u, v) = (u0, v0)  <=>  (K - s) u = (alpha u0 + tau v0) / tau^2,
 *     v = (alpha u + u0) / tau,  K = div(c^2 grad .),  s = (alpha / tau)^2.
 *
 * Calling sequence:
 *     hx_plan_create -> hx_plan_add (one or more instances) -> hx_plan_query
 *     -> hx_plan_bind (caller-allocated device arena) -> hx_plan_build
 *     -> hx_step (any number of times) -> hx_plan_destroy.
 *
 * Memory ownership: the plan owns host metadata only.  All device memory is
 * passed in by the caller: the arena (operators, index maps and the
 * per-step intermediates; must outlive the plan's use), the build workspace
 * (only during hx_plan_build) and the state buffers.  hx_step allocates
 * nothing; hx_plan_build may let rocBLAS/rocSOLVER allocate transient
 * device memory of their own during the build.
 *
 * State layout (one instance, nrhs right-hand sides): FP64, real,
 *     state[rhs][field][element][j][i],   fields (u, v) for the wave
 *     equation, (v1, v2, eta) for shallow water,
 * element e = ex + nex*ey, interior node (i, j), 1 <= i, j <= p-2, of the
 * element's p x p Chebyshev-Lobatto grid (ascending coordinates, x index
 * fastest).  Only interior nodes carry state; interface values follow from
 * flux continuity and the outer boundary is fixed at zero.
 *
 * Errors: every call returns an hx_status; negative values are errors and
 * a readable message is available from hx_last_error() on the calling
 * thread.  On any error before work is enqueued, device memory (arena,
 * state) is left untouched.
 */
#ifndef HPSEXP_H
#define HPSEXP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hx_plan hx_plan;

typedef enum {
  HX_OK = 0,
  HX_EINVAL = -1,     /* invalid argument or inconsistent input          */
  HX_ENOMEM = -2,     /* arena or workspace smaller than required        */
  HX_ESINGULAR = -3,  /* a leaf or merge system is singular (resonant pole) */
  HX_EUNSTABLE = -4,  /* max |R(ix)| on the real line exceeds 1 + tol     */
  HX_EDEVICE = -5,    /* a HIP / rocBLAS / rocSOLVER call failed          */
  HX_ESTATE = -6,     /* non-finite values in the state (check flag set)  */
  HX_ESTAGE = -7      /* call out of order (e.g. step before build)       */
} hx_status;

/* Problem kinds.
 * HX_WAVE_DIRICHLET: u_t = v, v_t = div(c^2 grad u), u = 0 on the boundary;
 *   state fields (u, v).
 * HX_SW_SLIP: linearised rotating shallow water (section 2.1, example 1)
 *   v_t = -f J v + c grad(eta), eta_t = c div(v), c = sqrt(gH), with slip
 *   walls n . v = 0; state fields (v1, v2, eta).  Each resolvent solves
 *   (Lap - s/c^2) eta = (s/(c^2 a)) eta0' + div(v0')/c - (f/(c a)) curl(v0')
 *   (a = alpha/tau, s = a^2 + f^2, primes: divided by tau) with the oblique
 *   wall condition a d_n eta - f d_t eta = (a n.v0' - f t.v0')/c, then
 *   v = (a - f J)(c grad(eta) - v0')/s.  Shallow-water instances run the
 *   matrix-core sweeps for any nrhs (HX_FLAG_UNBATCHED does not apply).
 *   In the precision form the wall rows join the FP64 residual, and the
 *   correction sweep's root system takes their residual. */
#define HX_WAVE_DIRICHLET 0
#define HX_SW_SLIP 1

/* Arithmetic of the stored operators and sweeps.
 * HX_FP64: operators, sweeps and pole sum in FP64.
 * HX_FP32_REFINE: the precision form.  Operators are built in FP64 and
 *   stored in FP32; each step runs one FP32 sweep per pole, the FP64
 *   residual of the collocation equations (interior rows and the flux
 *   jumps across element edges), one FP32 correction sweep on that
 *   residual, and the FP64 pole sum of the corrected solutions. */
#define HX_FP64 0
#define HX_FP32_REFINE 1

/* Plan flags (hx_plan_create). */
#define HX_FLAG_ALLOW_UNSTABLE 0x1u /* accept max|R(ix)| > 1 + 1e-6        */
#define HX_FLAG_NO_GRAPH       0x2u /* launch kernels eagerly, no hipGraph  */
#define HX_FLAG_CHECK_STATE    0x4u /* hx_step rejects non-finite states    */
#define HX_FLAG_UNBATCHED      0x8u /* one pass per right-hand side instead of
                                       batching them on the matrix cores
                                       (reference for the batching speedup)  */
#define HX_FLAG_AUTOTUNE       0x10u /* hx_plan_build times each batched
                                        instance's stages in each candidate
                                        shape (one or two right-hand-side
                                        tiles per block; merges also one-wave
                                        blocks, pole groups and fused level
                                        pairs; the upward
                                        element sweep also source staging)
                                        and keeps the fastest (hx_plan_tiles,
                                        hx_plan_variants)                    */
#define HX_FLAG_FUSED_MERGES   0x20u /* run the lowest merge levels in fused
                                        pairs, the level between them kept in
                                        LDS (the autotuner, when also set,
                                        may still choose otherwise)          */

/* Mesh: [x0,x1] x [y0,y1] split into nex x ney equal elements, each with a
 * p x p Chebyshev-Lobatto grid (section 2.2).  nex and ney are powers of
 * two (the merge tree pairs neighbours); 4 <= p <= 18. */
typedef struct {
  int nex, ney, p;
  double x0, x1, y0, y1;
} hx_mesh;

/* Coefficients.  kind = HX_WAVE_DIRICHLET: c2 is a host pointer to
 * nex*ney*p*p doubles, c(x)^2 at every node of every element
 * (element-major, local node i + p*j), finite and > 0, copied by
 * hx_plan_add (the caller keeps ownership); f and gH are ignored.
 * kind = HX_SW_SLIP: f (Coriolis frequency, any real) and gH (> 0) are
 * used, c2 is ignored (may be null). */
typedef struct {
  int kind;
  const double* c2;
  double f, gH;
} hx_coeffs;

/* Rational function R(z) = sum_{m=-M}^{M} b_m / (z - alpha_m) (eq.
 * def_RM).  npoles = 2M+1; alpha and b: host pointers to 2*npoles doubles,
 * interleaved (re, im), ordered m = -M..M.  Required: alpha_{-m} =
 * conj(alpha_m), b_{-m} = conj(b_m) (to 1e-12 relative), Re(alpha_m) != 0.
 * The symmetry lets real data use only m >= 0 (section 3.3, eq.
 * conjugate-matrix-inverses). */
typedef struct {
  int npoles;
  const double* alpha;
  const double* b;
} hx_rational;

/* Sizes and properties of a plan (hx_plan_query). */
typedef struct {
  size_t arena_bytes;          /* device bytes hx_plan_bind needs          */
  size_t operator_bytes;       /* of which stored solve-stage operators    */
  size_t workspace_bytes;      /* build workspace that builds all poles at once
                                  (capped at 16 GiB)                         */
  size_t workspace_min_bytes;  /* smallest workable build workspace        */
  long long dof_state;         /* fields * interior nodes * nrhs, summed   */
  long long dof_nodes;         /* fields * p*p nodes * elements * nrhs     */
  int folded_poles;            /* M+1, summed over instances                */
  int n_instances;
  double op_bytes_per_step;    /* stored operator bytes one step reads     */
  double flops_per_step;       /* 8 flops per complex multiply-add          */
  double max_abs_R;            /* max over instances of max |R(ix)|         */
  double fit_X;                /* min over instances of the checked X       */
  double sum_abs_b;            /* max over instances of sum |b_m|           */
} hx_info;

/* Creates an empty plan for device `device` (a HIP ordinal).  precision:
 * HX_FP64 or HX_FP32_REFINE.  flags: HX_FLAG_*.  Touches no device state.
 * HX_EINVAL on a bad precision or a null `out`. */
hx_status hx_plan_create(hx_plan** out, int precision, int device, unsigned flags);

/* Adds one problem instance (mesh, coefficients, step tau, requested
 * accuracy delta, rational function, number of right-hand sides) to a plan
 * that is not bound yet (section 1.2: fix tau, delta and R, then build the
 * 2M+1 solution operators once).  delta is used to check the supplied R:
 * fit_X is the largest X with |R(ix) - e^{ix}| <= delta on [-X, X]
 * (eq. RM_prop1), and max |R(ix)| over the real line must not exceed
 * 1 + 1e-6 (eq. RM_prop2) unless HX_FLAG_ALLOW_UNSTABLE.
 * instance_id (may be null) receives the instance's index, which is also
 * the position of its state pointer in hx_step.
 * HX_EINVAL: bad mesh / coefficients / tau / symmetry / nrhs < 1;
 * HX_EUNSTABLE: modulus check failed; HX_ESTAGE: plan already bound. */
hx_status hx_plan_add(hx_plan* plan, const hx_mesh* mesh, const hx_coeffs* coeffs,
                      double tau, double delta, const hx_rational* rational,
                      int nrhs, int* instance_id);

/* Fills *info.  Valid any time after the first hx_plan_add. */
hx_status hx_plan_query(const hx_plan* plan, hx_info* info);

/* Binds a device buffer of at least info.arena_bytes bytes, 256-byte
 * aligned, that the caller keeps alive while the plan is used.  Freezes
 * the plan (no more hx_plan_add).  HX_ENOMEM if too small, HX_EINVAL if
 * null or misaligned. */
hx_status hx_plan_bind(hx_plan* plan, void* arena, size_t arena_bytes);

/* Build stage (sections 1.3 and 2.3): for every instance and folded pole,
 * the element solution operators and the merge-tree operators, in FP64 on
 * the device.  workspace: device buffer of workspace_bytes >=
 * info.workspace_min_bytes (more bytes = more poles per batch).  stream: a
 * hipStream_t (null = default stream).  Synchronous: returns when the
 * operators are in the arena.  HX_ESINGULAR if a leaf or merge system is
 * singular, HX_ENOMEM if the workspace is too small, HX_EDEVICE on a
 * library failure, HX_ESTAGE if not bound. */
hx_status hx_plan_build(hx_plan* plan, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Advances every instance by n_steps steps of tau, in place:
 *     (u, v) <- R(tau L) (u, v)   (section 1.2; repetition eq. exp(n tau L)).
 * states[k]: device pointer to instance k's state (layout above).
 * stream: a hipStream_t (null = default).  Asynchronous (stream-ordered)
 * unless HX_FLAG_CHECK_STATE is set, in which case the states are checked
 * for non-finite values first (HX_ESTATE, states untouched).  n_steps == 0
 * is a no-op.  HX_ESTAGE if not built, HX_EINVAL on null pointers or
 * n_steps < 0. */
hx_status hx_step(hx_plan* plan, double* const* states, int n_steps, void* stream);

/* Kernel classes reported by hx_step_profile. */
#define HX_K_LEAF_UP    0  /* element upward pass: right-hand side, W g, N_i w   */
#define HX_K_MERGE_UP   1  /* merge upward pass, one launch per tree level       */
#define HX_K_MERGE_DOWN 2  /* merge downward pass, one launch per tree level     */
#define HX_K_LEAF_DOWN  3  /* element downward pass: w - S u_e                   */
#define HX_K_POLE_SUM   4  /* FP64 pole sum and velocity post-map (one RHS)       */
#define HX_K_RESIDUAL   5  /* FP64 residual of the precision form                 */
#define HX_K_SW_PREP    6  /* shallow water: eta, div v, curl v and wall values   */
#define HX_K_SW_ROOT    7  /* shallow water: root wall system                     */
#define HX_K_CLASSES    8

/* Diagnostic twin of hx_step: the same kernels, launched eagerly on
 * `stream` with a HIP event pair around every launch.  kernel_ms[c] and
 * launches[c] (arrays of n_classes entries, host) receive the summed
 * duration in milliseconds and the launch count of kernel class c.
 * Synchronous.  Errors as hx_step. */
hx_status hx_step_profile(hx_plan* plan, double* const* states, int n_steps, void* stream,
                          double* kernel_ms, int* launches, int n_classes);

/* Stages whose right-hand-side tile count (1 or 2 tiles of 16 columns per
 * block) is chosen per instance, by the default rule (2 when nrhs > 16)
 * or by the autotuner. */
#define HX_STAGE_LEAF_UP    0  /* element upward pass                          */
#define HX_STAGE_MERGE_UP   1  /* merge upward passes                          */
#define HX_STAGE_ROOT       2  /* shallow-water root system                    */
#define HX_STAGE_MERGE_DOWN 3  /* merge downward passes                        */
#define HX_STAGE_LEAF_DOWN  4  /* element downward pass (and fused pole sum)   */
#define HX_STAGES           5

/* Tile counts in use for instance `instance`: tiles[s] for the first
 * min(n, HX_STAGES) stages (host array).  0 for an instance that runs one
 * pass per right-hand side.  HX_EINVAL for a bad instance id. */
hx_status hx_plan_tiles(const hx_plan* plan, int instance, int* tiles, int n);

/* Kernel variants in use for instance `instance` (host array, first
 * min(n, HX_STAGES) stages), chosen by the default rules or the autotuner:
 *   HX_STAGE_LEAF_UP: 1 when the first upward sweep stages its source fields
 *     in LDS once per block and walks a group of poles, 0 when every block
 *     reads them for one pole;
 *   HX_STAGE_MERGE_UP / HX_STAGE_MERGE_DOWN: bit 0 set when every level
 *     runs one-wave (16-row) blocks, clear for the level rule (one wave
 *     where the level's rows fit one 16-row tile, else four waves, 64
 *     rows); HX_STAGE_MERGE_UP also bit 1, set when every block serves
 *     one pole, clear when the blocks of levels with many boxes walk a
 *     group of poles; bit 2 set when the lowest levels run in fused pairs
 *     (the level between them kept in LDS), clear when every level runs
 *     its own launch;
 *   other stages: 0.
 * All 0 for an instance that runs one pass per right-hand side.  Every
 * variant gives bit-identical results.  HX_EINVAL for a bad instance id. */
hx_status hx_plan_variants(const hx_plan* plan, int instance, int* variants, int n);

/* Name of a status code. */
const char* hx_status_str(int status);

/* Message of the last error on the calling thread ("" if none). */
const char* hx_last_error(void);

/* Destroys the plan's host objects (never frees caller memory). */
void hx_plan_destroy(hx_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* HPSEXP_H */
