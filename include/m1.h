/*
 * m1.h -- C ABI of the MI355X (gfx950) implicit M1 radiative-transfer multigrid solver.
 *
 * Method: H. Bloch, P. Tremblin, M. Gonzalez, E. Audit, "Towards a multigrid
 * method for the M1 model for radiative transfer" (arXiv 2208.14703).
 *   - unknowns: gray radiative energy E, flux F = (Fx, Fy) and gas temperature T
 *     (moments and M1 closure, Sect. 2.1);
 *   - one implicit Euler step with the HLL flux at wave speeds +-c (Rusanov),
 *     Sect. 2.2, extended to 2-D by directions, with absorption (sigma_a),
 *     emission (a_r T^4), scattering (sigma_s) and gas energy C_v T implicit in
 *     the diagonal block (the source terms of the moment system, Sect. 2.1);
 *   - solved by the nonlinear FAS multigrid of Sect. 4 / Appendix A: Jacobi
 *     smoothing on the finest level (Algorithm 1), full-weighting restriction
 *     and linear prolongation (Sect. 4.2), coarse problems in pseudo-time with
 *     explicit sub-steps and an implicit Jacobi step (Algorithm 3), the
 *     admissibility-restoring correction (eq. prolongatedSol), and relative
 *     residual stopping with pseudo-time step adaptation.
 *
 * Conventions for every entry point:
 *   - all array pointers are HIP DEVICE pointers owned by the caller; fields are
 *     separate arrays of nx*ny doubles, row-major with x fastest (cell (i,j) at
 *     j*nx + i); in 1-D ny == 1 and Fy must be NULL;
 *   - every call enqueues on the plan's stream; only m1_step, m1_residual,
 *     m1_sync and the batch wait/poll calls block the host;
 *   - no entry point allocates device memory: m1_plan_create carves the
 *     caller-provided workspace; the plan itself is a small host object;
 *   - argument errors are detected on the host, return immediately and enqueue
 *     nothing; no C++ exception crosses the ABI;
 *   - a plan is bound to one stream and is not thread-safe.
 */
#ifndef M1_H
#define M1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    M1_OK = 0,
    M1_ERR_ARG = 1,             /* invalid argument (detected on the host, nothing enqueued) */
    M1_ERR_NOT_ADMISSIBLE = 2,  /* input state has E <= 0, T <= 0, |F| > cE or a non-finite value */
    M1_ERR_NO_CONVERGENCE = 3,  /* max_cycles reached; the state holds the last (admissible) iterate */
    M1_ERR_WORKSPACE = 4,       /* workspace NULL, misaligned or smaller than m1_workspace_bytes() */
    M1_ERR_DEVICE = 5,          /* a HIP runtime call failed */
    M1_ERR_BUSY = 6,            /* engine queue full / request still running */
    M1_ERR_BUDGET = 7           /* request larger than the engine's HBM budget */
} m1_status;

typedef enum {
    M1_BC_PERIODIC = 0,
    M1_BC_REFLECTIVE = 1,
    M1_BC_NEUMANN = 2,
    M1_BC_DIRICHLET = 3,
    M1_BC_INFLOW = 4
} m1_bc_kind;
typedef enum { M1_FP64 = 0, M1_MIXED = 1 } m1_precision;
typedef enum { M1_DTAU_SIGNED = 0, M1_DTAU_LITERAL = 1 } m1_dtau_rule;
typedef enum { M1_SMOOTH_JACOBI = 0, M1_SMOOTH_RBGS = 1 } m1_smoother;
typedef enum { M1_CYCLE_V = 0, M1_CYCLE_W = 1, M1_CYCLE_F = 2 } m1_cycle;
typedef enum { M1_TRANSFER_FULL = 0, M1_TRANSFER_MEAN = 1 } m1_transfer;

/* Boundary condition of one side.  Ghost state of the neighbour outside the
 * domain: PERIODIC wraps; REFLECTIVE mirrors the adjacent cell with its normal
 * flux negated; NEUMANN copies the adjacent cell; DIRICHLET uses (E, Fx, Fy),
 * which must be admissible (|F| <= cE up to a relative 1e-12); INFLOW uses
 * (E, Fx, Fy) for the boundary cells whose centres lie in [lo, hi] (fractions
 * of the side's length from its low-coordinate end, 0 <= lo <= hi <= 1: cell a
 * of n when lo n <= a + 1/2 <= hi n) and the isotropic state (Eo > 0, F = 0)
 * elsewhere, on every level (a beam entering through part of a side into
 * ambient radiation, Sect. 5.1).  lo, hi and Eo are read for INFLOW only.  Periodic sides come in pairs (x-/x+,
 * y-/y+).                                                                    */
typedef struct {
    int32_t kind;
    int32_t pad_;
    double E, Fx, Fy;
    double lo, hi, Eo;
} m1_bc;

/* Discrete problem: the data of the implicit HLL system (Sect. 2.2) plus the
 * source coefficients.  dt is the physical step (CFL*h/c in the paper's
 * notation), hx/hy the cell sizes, c the light speed, a_r the radiation
 * constant, c_v the gas heat capacity per volume (> 0).
 * bc[] order: x-, x+, y-, y+ (y sides ignored in 1-D).  At most 2^29 cells
 * (nx*ny; e.g. 16384 x 16384 or 23170^2), so that every cell's byte offset in
 * an FP64 field fits 32 bits; larger grids are rejected with M1_ERR_ARG.    */
typedef struct {
    int32_t dim, nx, ny, pad_;
    double hx, hy, dt, c, a_r, c_v;
    m1_bc bc[4];
} m1_grid;

/* Solver parameters (m1_default_params gives the paper's: nu0 = 3, pseudo-time
 * steps m = 3, nu_l = 1, dtau_im0 = 1e-3).
 *   levels        total levels including the finest; 0 = coarsen while both
 *                 sides stay even and >= 4 (1 = plain Jacobi, Sect. 5.1);
 *   nu0           finest-level Jacobi sweeps before and after the correction;
 *   nu_l          Jacobi sweeps per implicit pseudo-time step (coarse levels);
 *   pseudo_steps  pseudo-time steps per coarse smoothing (Algorithm 3);
 *   sub_steps     max explicit sub-steps per pseudo-time step; each covers
 *                 eta times the remaining admissible length of its ray;
 *   max_cycles    V-cycles per time step before M1_ERR_NO_CONVERGENCE;
 *   dtau_rule     pseudo-time step adaptation: SIGNED (relative decrease of the
 *                 residual vs the previous cycle) or LITERAL (|change| / r0);
 *   pseudo_local  1: the implicit pseudo-time step of each cell uses the pseudo
 *                 time its explicit sub-steps reached (consistent steady state);
 *                 0: dtau_im in every cell;
 *   smoother      finest-level sweeps: M1_SMOOTH_JACOBI (Algorithm 1) or
 *                 M1_SMOOTH_RBGS, red-black nonlinear Gauss-Seidel (the
 *                 alternative of Sect. 6.3): the cells with i + j even take
 *                 the relaxed Jacobi update, then the others the update of
 *                 that state (FP64 plans only; not in engines);
 *   cycle         shape of the multigrid cycle: M1_CYCLE_V (Appendix A's
 *                 V-cycle), M1_CYCLE_W (each coarse problem below the finest
 *                 visited twice per visit of the level above) or M1_CYCLE_F
 *                 (an F-cycle of the coarse problem, then a V-cycle of it);
 *                 the alternatives of Sect. 6.3.  Every visit of a coarse
 *                 level runs the pseudo-time smoothing of Algorithm 3 before
 *                 and after its correction (the coarsest: once per visit).
 *                 W and F: not in engines;
 *   transfer      grid-transfer operators: M1_TRANSFER_FULL (Sect. 4.2: linear
 *                 prolongation, full-weighting restriction R = 2^-d P^T) or
 *                 M1_TRANSFER_MEAN (coarse cell I is fine cells 2I, 2I+1 per
 *                 axis: piecewise-constant prolongation and R = 2^-d P^T, the
 *                 mean of the 2^d children; Sect. 6.3 leaves the operators
 *                 open).  Also restricts the coarse opacities.  MEAN: FP64
 *                 plans only, not in engines;
 *   precision     M1_FP64 or M1_MIXED (FP32 delta-form smoothing and coarse
 *                 levels, FP64 residual, projection and T^4 update; M1_MIXED
 *                 requires nu_l = 1: its coarse steps fuse one sweep);
 *   dtau_carry    1 (default): dtau_im runs on from one time step into the
 *                 next within a call (Algorithm 4, the overall algorithm of
 *                 Appendix A, does not set it at the start of a time step;
 *                 Sect. 5 gives its initial value); 0: it restarts at dtau_im0
 *                 at every time step.  A call always starts at dtau_im0; m1_info.dtau
 *                 gives the value to start the next call with;
 *   dtau_im0      initial implicit pseudo-time step (Sect. 5: 1e-3);
 *   eps_inc/dec   adaptation thresholds (x1.1 above eps_inc, /2 below eps_dec);
 *   eta           fraction of the admissible ray used (sub-steps, projection);
 *   rtol          stop when |b - A(v)| <= rtol |b - A(v^n)|;
 *   dtau_min/max  clamp of dtau_im;
 *   omega         relaxation of the finest-level sweeps: u <- u + omega (J(u) - u);
 *                 1 is Algorithm 1, 0 < omega <= 1 keeps admissibility.      */
typedef struct {
    int32_t levels, nu0, nu_l, pseudo_steps, sub_steps, max_cycles, dtau_rule, pseudo_local, precision, smoother;
    int32_t cycle, transfer, dtau_carry, pad_;
    double dtau_im0, eps_inc, eps_dec, eta, rtol, dtau_min, dtau_max, omega;
} m1_params;

/* State (E, Fx, Fy, T), device pointers, nx*ny each; Fy == NULL in 1-D. */
typedef struct {
    double *E, *Fx, *Fy, *T;
} m1_state;

/* Opacities per cell (>= 0, finite), device pointers; must outlive the plan. */
typedef struct {
    const double *sigma_a, *sigma_s;
} m1_opacity;

/* Result of m1_step.  cycles: total V-cycles over all steps; rel_residual and
 * r0: of the last step; first_bad_cell: index of the first non-admissible
 * input cell (or -1); status: as returned; stalled_cells: pseudo-time
 * stalls over the call (m1_step, m1_step3; 0 elsewhere): coarse-level cell
 * updates whose explicit sub-steps could not move because the state lies on
 * the boundary of the admissible set and the source points out of it
 * (tau* = 0 in Algorithm 3), so that the pseudo-time step left the cell
 * unchanged.                                                                 */
typedef struct {
    int32_t cycles, status, levels, steps_done;
    double r0, rel_residual, dtau;
    int64_t first_bad_cell;
    int64_t stalled_cells;
} m1_info;

typedef struct m1_plan m1_plan;

const char* m1_strerror(m1_status s);

/* Fill p with the paper's parameters (see m1_params). */
void m1_default_params(m1_params* p);

/* Bytes of device workspace a plan needs (0 on invalid arguments): the
 * per-level storage of the FAS scheme (Sect. 4.2: on every coarse level the
 * restricted state, the iterate, the right-hand side of the coarse problem,
 * its residual and the opacities; Sect. 5.1 notes that these auxiliary
 * vectors make the multigrid's memory grow with the number of levels), plus
 * the finest level's right-hand side, partner state and residual, and (mixed
 * precision) the FP32 copies.                                                 */
size_t m1_workspace_bytes(const m1_grid* g, const m1_params* p);

/* Build the level hierarchy of Sect. 4.2 (each level halves both sides,
 * spacing 2^l h; `levels` of them, or down to side 4) with coarse opacities
 * by full weighting of the fine ones, inside `workspace` (device memory,
 * 256-byte aligned, at least m1_workspace_bytes bytes).  `stream` is a
 * hipStream_t (NULL = default).  Opacities are validated (M1_ERR_ARG if
 * negative or non-finite).  The plan keeps pointers to `op` arrays and
 * `workspace`; both must outlive it.  Returns M1_ERR_WORKSPACE for a missing,
 * misaligned or short workspace; writes *out only on M1_OK.                 */
m1_status m1_plan_create(const m1_grid* g, const m1_params* p, const m1_opacity* op, void* workspace,
                         size_t workspace_bytes, void* stream, m1_plan** out);
void m1_plan_destroy(m1_plan* plan);
int32_t m1_plan_levels(const m1_plan* plan);
m1_status m1_level_dims(const m1_plan* plan, int32_t level, int32_t* nx, int32_t* ny);

/* Residual of eq. (defResidual) on the finest level, r = b - A(v) with
 * b = (E^n, F^n, C_v T^n) taken from `vn`.  Writes the discrete L2 norm of
 * (r_E, r_Fx/c, r_Fy/c, r_T) to *norm_out (host pointer; blocks), and the
 * residual fields to r_out when it is not NULL.                              */
m1_status m1_residual(m1_plan* plan, const m1_state* v, const m1_state* vn, double* norm_out, m1_state* r_out);

/* One V-cycle of the overall algorithm (Appendix A, Algorithm 4: nu0 finest
 * Jacobi sweeps, the FAS coarse problems of Sect. 4.2 in pseudo-time,
 * Algorithm 3, the corrections of eq. prolongatedSol, nu0 sweeps again) of the
 * time step whose initial state is `vn`, updating the iterate `v` in place,
 * with implicit pseudo-time step dtau (> 0).  v must not alias vn.
 * info == NULL: asynchronous (enqueued on the plan's stream).  Otherwise the
 * call blocks and fills *info: cycles = 1, levels, dtau, r0 = |b - A(vn)| and
 * rel_residual = |b - A(v)| / r0 of the updated iterate (norm of
 * m1_residual; 0 when r0 = 0), status M1_OK.                                */
m1_status m1_vcycle(m1_plan* plan, m1_state* v, const m1_state* vn, double dtau, m1_info* info);

/* nsteps implicit Euler steps (the overall algorithm of Appendix A,
 * Algorithm 4): v holds v^n on entry and v^{n+nsteps} on exit.  Each step sets
 * b = (E^n, F^n, C_v T^n) and runs cycles until |b - A(v)| <= rtol |b - A(v^n)|
 * (the relative residual of Sect. 5), adapting dtau_im after every cycle
 * (x1.1 / 0.5 by eps_inc / eps_dec).  dtau_im starts at dtau_im0 and, with
 * dtau_carry, runs on from step to step; without it, every step restarts it.  Validates the
 * input state first: M1_ERR_NOT_ADMISSIBLE (info->first_bad_cell set, v
 * untouched) if a cell is outside S = {E > 0, |F| <= cE, T > 0}.
 * M1_ERR_NO_CONVERGENCE when a step reaches max_cycles (v then holds that
 * step's last, admissible iterate).  Blocks; info (host) may be NULL.        */
m1_status m1_step(m1_plan* plan, m1_state* v, int32_t nsteps, m1_info* info);

/* ---- allocation-free time steps ----------------------------------------------
 * For callers that cannot allocate device memory or pinned host memory (code
 * that must not call hipMalloc, hipHostMalloc or a framework allocator, such
 * as tight serving loops or harnesses that forbid allocation).
 * m1_step_static runs m1_step on a plan whose workspace is a static device
 * array of M1_STATIC_SCRATCH_BYTES bytes that the library holds on every
 * device it runs on until the process ends (its address is looked up with
 * hipGetSymbolAddress on the first call on each device).  It allocates no
 * device or pinned memory, records no graphs, and gives m1_step's results to
 * the bit.  The caller passes grid, parameters, opacity and state (device
 * arrays, as for m1_plan_create and m1_step) and the stream, which must
 * belong to the current device.  80 MiB hold a 2-D plan of up to about
 * 540 K cells in FP64 and 290 K cells in mixed precision (512 x 512: 39 and
 * 71 MiB); problems whose m1_workspace_bytes exceeds M1_STATIC_SCRATCH_BYTES
 * are rejected with M1_ERR_WORKSPACE, invalid arguments with M1_ERR_ARG;
 * otherwise as m1_step (blocks; info may be NULL).  Nothing in the array has
 * to start at zero: every buffer is written before it is read.  All calls on
 * one device share its array and a host slot: calls that overlap on one
 * device race (serialise them).                                             */
#define M1_STATIC_SCRATCH_BYTES (80u << 20)
m1_status m1_step_static(const m1_grid* g, const m1_params* p, const m1_opacity* op, m1_state* v, int32_t nsteps,
                         void* stream, m1_info* info);

/* ---- single operations of the cycle on one level (parity checks, custom drivers) ---- */

/* out = A_l(v) on level `level` (spacing 2^level h, opacities of that level). */
m1_status m1_apply_A(m1_plan* plan, int32_t level, const m1_state* v, m1_state* out);
/* One relaxed Jacobi sweep of A_0(u) = b on the finest level (Algorithm 1 with
 * weight omega from the plan's params): v_out = v_in + omega (J(v_in) - v_in). */
m1_status m1_sweep(m1_plan* plan, const m1_state* b, const m1_state* v_in, m1_state* v_out);
/* nsweeps >= 1 such sweeps from v_in into v_out (v_in is not written), as the
 * cycle runs them: two consecutive sweeps in one launch when the launch shape
 * "pair_rows" is on (2-D), which gives the one-by-one sweeps' result to the
 * bit.  v_out must not alias v_in or b.  Uses the plan's spare finest-level
 * state as the other buffer: not concurrently with m1_vcycle/m1_step on the
 * same plan.  M1_ERR_ARG for nsweeps < 1 or an invalid state. */
m1_status m1_sweeps(m1_plan* plan, const m1_state* b, const m1_state* v_in, m1_state* v_out, int32_t nsweeps);
/* One pseudo-time step (Algorithm 3) of M du/dtau + A_l(u) = f on level `level`
 * (level >= 1 in the cycle; any level accepted), from u_in to u_out.          */
m1_status m1_pseudo_step(m1_plan* plan, int32_t level, double dtau, const m1_state* f, const m1_state* u_in,
                         m1_state* u_out);
/* Restriction (Sect. 4.2: full weighting; with M1_TRANSFER_MEAN the 2^d-cell
 * mean) of a state from `level` to level+1.                                  */
m1_status m1_restrict(m1_plan* plan, int32_t level, const m1_state* fine, m1_state* coarse);
/* Residual of level `level` and its restriction, as the downward leg of a
 * V-cycle forms them (Appendix A, Algorithm 4): r = rhs - A_l(u) (eq.
 * defResidual, with the level's opacities and spacing), then the plan's
 * restriction (Sect. 4.2, eq. restrictionOperator, or the 2^d-cell mean) of u
 * into vc and of r into rc (level+1 arrays).  In 2-D with full weighting and
 * the launch shape "residual_restrict" on (default) r is never stored; otherwise it is written
 * to the plan's residual buffer of that level first (not concurrently with
 * m1_vcycle/m1_step on the same plan).  M1_ERR_ARG unless 0 <= level <
 * levels - 1.                                                                */
m1_status m1_residual_restrict(m1_plan* plan, int32_t level, const m1_state* u, const m1_state* rhs, m1_state* vc,
                               m1_state* rc);
/* Correction of `level` from level+1 with admissibility (eq. prolongatedSol):
 * w = u + P(uc - vc), P the plan's prolongation (linear, eq.
 * prolongationOperator, or piecewise constant); out = w where admissible,
 * else u + eta tau*(u, w-u) (w-u).
 * out may alias u.                                                           */
m1_status m1_prolong_project(m1_plan* plan, int32_t level, const m1_state* u, const m1_state* uc,
                             const m1_state* vc, m1_state* out);
/* Wait for all work enqueued on the plan's stream. */
m1_status m1_sync(m1_plan* plan);
/* Pseudo-time stalls (see m1_info.stalled_cells) counted on this plan since
 * its creation, its last m1_step or the last reset: *count (host; blocks),
 * then the counter is cleared when `reset` is nonzero.  Counts the coarse
 * cycle's pseudo-time steps and m1_pseudo_step.                              */
m1_status m1_stalls(m1_plan* plan, int64_t* count, int32_t reset);

/* ---- launch-shape settings ----------------------------------------------------
 * Process-wide settings of how the cycle is launched (environment variables
 * M1_SWEEP_ROWS, M1_PAIR_ROWS, M1_MX_SWEEP_ROWS, M1_RESIDUAL_RESTRICT, M1_TAIL_CELLS,
 * M1_TILED_MAX_CELLS, M1_GRAPHS, M1_BATCH_GRID give the initial values).  None of them changes any result: every launch
 * shape runs the same per-cell arithmetic.  Keys:
 *   "sweep_rows"       rows of the 64-wide tile of the LDS-staged finest-level
 *                      Jacobi sweep (2-D sweeps without the norm; 4, 8 or 16),
 *                      0 = one cell per thread without LDS (default 4; read at
 *                      each launch; engines read it when their tables are built);
 *   "pair_rows"        rows of the 64-wide tile of the kernels that run two
 *                      consecutive finest-level sweeps of a cycle (2-D, without
 *                      the norm; FP64 sweeps and mixed-precision correction
 *                      sweeps) in one launch, the first sweep's iterate kept in
 *                      LDS (4, 8 or 16); 0 = each sweep its own launch
 *                      (default 8; read at each launch);
 *   "mx_sweep_rows"    the same for the mixed-precision correction sweeps;
 *   "residual_restrict" 1: the finest-level residual of a cycle is restricted
 *                      to level 1 as it is formed, in one launch (2-D);
 *                      0: stored, then restricted (default 1; read at each
 *                      launch);
 *   "tail_cells"       levels of at most this many cells run in one workgroup
 *                      (default 256; read when a plan is created);
 *   "tiled_max_cells"  largest level whose smoothing legs run as one LDS-tiled
 *                      launch each (2-D, sides multiples of 16; default 65536;
 *                      0 = none; read when a plan is created);
 *   "graphs"           1: m1_step and engine rounds replay their V-cycles from
 *                      hipGraph recordings (made on first use per set of state
 *                      buffers, resp. once the engine's resident set has been
 *                      the same for a round); 0: launches are enqueued one by
 *                      one (default 0; read when a plan or engine is created);
 *   "batch_grid"       most blocks of one batched launch (default 16384; read
 *                      at each launch, and when a V-cycle is recorded);
 *   "stage3"           3-D plans: 0 one-cell stencil kernels only; 1 the
 *                      sweeps and A(u) of levels of at least 2^23 cells
 *                      staged in LDS per z-plane; 2 every stencil operation
 *                      staged where the level is at least 32 cells wide
 *                      (default 1; the same bits in every case; read at each
 *                      launch);
 *   "prolong3_lds"     3-D plans: 1 the correction of eq. prolongatedSol
 *                      with the coarse differences of a tile staged in LDS, 0
 *                      one fine cell per thread reading its coarse cells
 *                      (default 1; the same bits; read at each launch).
 * m1_tune_set: M1_ERR_ARG for an unknown key or a value out of range.
 * m1_tune_get: the current value, -1 for an unknown key.  The autotuner
 * (paper_2208_14703_amd/autotune.py) times candidates and stores its choice. */
m1_status m1_tune_set(const char* key, int64_t value);
int64_t m1_tune_get(const char* key);

/* ---- batched and served solves ------------------------------------------------
 * An engine advances many independent problems (requests) together.  Each
 * request is one 2-D problem (grid, opacity, state, number of implicit steps);
 * when admitted -- first come, first served, as soon as its workspace fits in
 * the engine's arena -- it gets its own plan carved from the arena.  All
 * admitted requests then run the same V-cycle: every level operation is ONE
 * launch over all of them (a work list of (request, 256-cell tile) entries),
 * the levels of at most 256 cells run as one workgroup per request, and every
 * request keeps its own pseudo-time step, residual norm and stopping test, so
 * its result equals the result of solving it alone.  A request's state stays
 * in its own device arrays, updated in place, across its steps; requests that
 * finish a step start the next one, finished requests free their workspace
 * and waiting ones are admitted between rounds (continuous batching).
 * Engine calls are serialised internally: submit/poll/cancel may be called from
 * other threads while one thread runs rounds. */
typedef struct m1_engine m1_engine;

/* Workspace one request of this grid takes from the engine arena. */
size_t m1_engine_request_bytes(const m1_grid* g, const m1_params* p);

/* Engine over `arena` (device memory, 256-byte aligned, `arena_bytes` long;
 * owned by the caller, must outlive the engine).  `p` fixes the smoothing
 * structure every request must share (nu0, pseudo_steps (odd), sub_steps,
 * pseudo_local, omega, eta, nu_l = 1, precision: M1_FP64 or M1_MIXED, each
 * request's result equal to the bit to its single-problem solve); per-request
 * tolerances (rtol, max_cycles, dtau settings) may differ.  At most
 * `max_requests` requests are resident at once.  stream: hipStream_t.        */
m1_status m1_engine_create(const m1_params* p, void* arena, size_t arena_bytes, int32_t max_requests, void* stream,
                           m1_engine** out);
void m1_engine_destroy(m1_engine* e);

/* Queue a request of `nsteps` implicit steps on state `v` (device arrays,
 * caller-owned, updated in place; v and the opacity must outlive the request).
 * p == NULL uses the engine's parameters.  M1_ERR_BUDGET if the request can
 * never fit in the arena, M1_ERR_ARG if it is not 2-D, not compatible, or
 * larger than 2^28 cells (2^20 work tiles of its finest level).             */
m1_status m1_batch_submit(m1_engine* e, const m1_grid* g, const m1_params* p, const m1_opacity* op, m1_state* v,
                          int32_t nsteps, uint64_t* ticket);
/* One round: admit waiting requests that fit, start pending time steps, run
 * `cycles` V-cycles of every resident request, retire finished steps and
 * requests.  Blocks until the round's work is done.                          */
m1_status m1_batch_run(m1_engine* e, int32_t cycles, int32_t* n_running, int32_t* n_pending);
/* M1_OK and the request's result in *info once it is done, M1_ERR_BUSY while
 * it is queued or running.                                                   */
m1_status m1_batch_poll(m1_engine* e, uint64_t ticket, m1_info* info);
/* Wait until the request is done and return its final status: while the
 * serving loop runs, sleep until it finishes the request; otherwise run
 * rounds (4 V-cycles each) on the calling thread.  info may be NULL.         */
m1_status m1_batch_wait(m1_engine* e, uint64_t ticket, m1_info* info);
/* Drop a queued or running request at the next round boundary (its state is
 * left at its last admissible iterate).                                      */
m1_status m1_batch_cancel(m1_engine* e, uint64_t ticket);
/* Host steady-clock times (s) of submission, admission and completion.       */
m1_status m1_batch_times(m1_engine* e, uint64_t ticket, double* t_submit, double* t_admit, double* t_done);
/* Forget a finished request (frees its host record).                         */
m1_status m1_batch_release(m1_engine* e, uint64_t ticket);

/* HBM of the engine's request pool (the part of the arena that request
 * workspaces are carved from; the rest holds the device tables): bytes in use
 * and in total, and the numbers of resident and waiting requests (either
 * pointer may be NULL).  Does not wait for a running round: the figures are
 * those of the last admission or retirement.                                 */
m1_status m1_engine_memory(m1_engine* e, size_t* pool_in_use, size_t* pool_bytes, int32_t* resident,
                           int32_t* pending);

/* Serving loop (continuous batching without a driving caller).  Starts one
 * host thread of the library that runs rounds of `cycles` V-cycles as long as
 * requests are resident or waiting and sleeps while the engine is empty, so
 * requests submitted from any thread while others are on the GPU are admitted
 * as memory and slots free up.  Clients only submit, then poll or wait.
 * M1_ERR_BUSY if a loop is already started (or ended on an error and has not
 * been stopped); M1_ERR_ARG for cycles < 1.                                  */
m1_status m1_serve_start(m1_engine* e, int32_t cycles);
/* Stop the serving loop after its current round and join its thread (no-op
 * if none).  Requests not yet done stay in the engine; a later
 * m1_serve_start or m1_batch_run continues them.  Returns the first error the
 * loop met (its rounds stop at the first error), else M1_OK.  Also called by
 * m1_engine_destroy.                                                         */
m1_status m1_serve_stop(m1_engine* e);

/* ---- three dimensions ---------------------------------------------------------
 * The method with d = 3: the paper writes its scheme in 1-D and says the
 * extension to higher dimensions is direct (Sect. 2.2); its restriction is
 * R = 2^-d P^T with d = 1, 2, 3 (Sect. 4.2).  Per axis the left/right operators
 * of Sect. 3.1 with the directional flux (F_axis, c^2 P[., axis]) of the 3-D
 * closure (Sect. 2.1), the implicit sources, the nonlinear Jacobi sweep
 * (Algorithm 1), pseudo-time steps (Algorithm 3), the admissible correction
 * (eq. prolongatedSol), trilinear prolongation with full weighting R, and the
 * V-cycle / time-step driver of Appendix A, with the W- and F-cycles of
 * Sect. 6.3 as the 2-D plans run them.  FP64 plans with full weighting, Jacobi
 * smoothing and nu_l = 1 (other m1_params choices give M1_ERR_ARG); sides
 * PERIODIC, REFLECTIVE, NEUMANN or DIRICHLET. */

/* Side condition of a 3-D grid (kinds as m1_bc; (E, Fx, Fy, Fz) for DIRICHLET). */
typedef struct {
    int32_t kind;
    int32_t pad_;
    double E, Fx, Fy, Fz;
} m1_bc3;

/* 3-D discrete problem: nx*ny*nz cells (at most 2^29), cell sizes hx, hy, hz,
 * the other data as m1_grid.  bc[] order: x-, x+, y-, y+, z-, z+.            */
typedef struct {
    int32_t nx, ny, nz, pad_;
    double hx, hy, hz, dt, c, a_r, c_v;
    m1_bc3 bc[6];
} m1_grid3;

/* 3-D state (E, Fx, Fy, Fz, T), device pointers, nx*ny*nz each, x fastest
 * (cell (i, j, k) at (k ny + j) nx + i).  Opacities: m1_opacity over the same
 * cells.                                                                      */
typedef struct {
    double *E, *Fx, *Fy, *Fz, *T;
} m1_state3;

typedef struct m1_plan3 m1_plan3;

/* Bytes of device workspace of a 3-D plan (0 on invalid arguments): per coarse
 * level the restricted state, two iterates, the FAS right-hand side, the
 * residual and the opacities (Sect. 4.2); on the finest level the right-hand
 * side, a partner state and the residual.                                   */
size_t m1_workspace3_bytes(const m1_grid3* g, const m1_params* p);
/* Hierarchy of Sect. 4.2 in 3-D: every side halved per level while all stay
 * even and >= 8 (or `levels` levels), coarse opacities by full weighting;
 * buffers carved from `workspace` (device, 256-byte aligned).  Opacities
 * validated (M1_ERR_ARG if negative or non-finite); M1_ERR_WORKSPACE for a
 * missing, misaligned or short workspace; `op` arrays and `workspace` must
 * outlive the plan.                                                         */
m1_status m1_plan3_create(const m1_grid3* g, const m1_params* p, const m1_opacity* op, void* workspace,
                          size_t workspace_bytes, void* stream, m1_plan3** out);
void m1_plan3_destroy(m1_plan3* plan);
int32_t m1_plan3_levels(const m1_plan3* plan);
m1_status m1_level3_dims(const m1_plan3* plan, int32_t level, int32_t* nx, int32_t* ny, int32_t* nz);
/* out = A_l(v) on `level` (Sect. 3.1 with the implicit sources). */
m1_status m1_apply3(m1_plan3* plan, int32_t level, const m1_state3* v, m1_state3* out);
/* One relaxed Jacobi sweep (Algorithm 1) of A(u) = b on the finest level; v_out
 * must not alias v_in.                                                        */
m1_status m1_sweep3(m1_plan3* plan, const m1_state3* b, const m1_state3* v_in, m1_state3* v_out);
/* One pseudo-time step (Algorithm 3) of M du/dtau + A_l(u) = f on `level`. */
m1_status m1_pseudo_step3(m1_plan3* plan, int32_t level, double dtau, const m1_state3* f, const m1_state3* u_in,
                          m1_state3* u_out);
/* Full-weighting restriction (R = 2^-3 P^T) from `level` to level+1. */
m1_status m1_restrict3(m1_plan3* plan, int32_t level, const m1_state3* fine, m1_state3* coarse);
/* out = u + P(uc - vc) on `level` (trilinear P) with the admissibility
 * correction of eq. prolongatedSol; out may alias u.                         */
m1_status m1_prolong_project3(m1_plan3* plan, int32_t level, const m1_state3* u, const m1_state3* uc,
                              const m1_state3* vc, m1_state3* out);
/* r = b - A(v), b = (E^n, F^n, C_v T^n) of vn; the L2 norm of (r_E, r_F/c, r_T)
 * to *norm_out (host; blocks), the fields to r_out when not NULL.            */
m1_status m1_residual3(m1_plan3* plan, const m1_state3* v, const m1_state3* vn, double* norm_out, m1_state3* r_out);
/* One cycle of the plan's shape (params.cycle: Appendix A's V-cycle, or the W- or F-cycle of Sect. 6.3) of
 * A(v) = b(vn) with pseudo-time step dtau, in place on v (v must not alias vn). */
m1_status m1_vcycle3(m1_plan3* plan, m1_state3* v, const m1_state3* vn, double dtau);
/* nsteps implicit Euler steps in place on v (Appendix A, Algorithm 4), as m1_step: cycles until the relative
 * residual rtol or A's rounding level, dtau carried from step to step (dtau_carry) and adapted after every cycle; M1_ERR_NOT_ADMISSIBLE
 * for a non-admissible input (info->first_bad_cell), M1_ERR_NO_CONVERGENCE after max_cycles.                   */
m1_status m1_step3(m1_plan3* plan, m1_state3* v, int32_t nsteps, m1_info* info);

#ifdef __cplusplus
}
#endif
#endif /* M1_H */
