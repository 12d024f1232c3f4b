/* libsisph: the per-timestep hot path of the simple iterative ISPH (SISPH)
 * scheme of Muta, Ramachandran & Negi (arXiv:1908.01762) on one AMD MI355X
 * (gfx950).
 *
 * One SISPH time step (Algorithm 1, section 3.1) is split the way the
 * paper's implementation notes split it into two stages (section 3.3):
 *
 *   sisph_bin       cell binning of the particles at r^n and the neighbour
 *                   sets N^n = { j : |r_ij|^2 < R^2 } (R = kernel support),
 *                   and with them the summation density
 *                   (eq. summation_density) and free-surface flags
 *                   (section 3)
 *   sisph_predict   wall ghost velocity (eqs. vf,
 *                   vg-adami, vg-no-normal), predictor accelerations
 *                   (eqs. mom:sph:visc, mom:sph:av, mom:sph:gtvf:stress, body
 *                   force), r* and u* (eqs. int:rnp1, int:vint), then the
 *                   binning and neighbour sets N* at r*, and the wall u*
 *   sisph_ppe_solve PPE right-hand side and coefficients (eqs. sph-ppe,
 *                   coeff, coeff1), the damped-Jacobi iteration
 *                   (eq. p-sor) with the wall pressure of eq. p-shepard
 *                   re-extrapolated before every sweep, and the convergence
 *                   test of eq. convergence (min 2 sweeps)
 *   sisph_correct   pressure acceleration (eq. mom:sph:press:pij or
 *                   mom:sph:press:symm) and u^{n+1} (eq. int:vnp1), K GTVF
 *                   sub-steps on the frozen N* (eqs. mom:sph:gtvf,
 *                   int:gtvf:pos, int:gtvf:vel:tmp), the transport velocity
 *                   and the position update (eqs. int:vhatnp2, int:rnp2)
 *   sisph_step      all four, nsteps times
 *
 * Units are SI.  Arrays crossing this boundary are host memory, float64,
 * row-major [n][dim], in the caller's original particle order with fluid
 * rows first and wall rows after them.  The device workspace is device
 * memory owned by the caller (for instance a torch uint8 tensor); the
 * library sub-allocates it and never frees it.  A context is not
 * thread-safe; distinct contexts on distinct streams are independent.
 * Work is queued on the context's stream and a call may return before its
 * last kernels finish (sisph_correct; the settle of the final iterate at
 * the end of sisph_ppe_solve once its reference pressure is set, for a
 * case solved in one persistent launch); calls that return host data wait
 * for the stream, so the workspace is consistent only after such a call or
 * a synchronisation of the stream.
 * Every function returns a status code and never throws.
 */
#ifndef SISPH_H
#define SISPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    SISPH_OK = 0,
    SISPH_WARN_MAXITER = 1,   /* PPE stopped at max_iter; fields valid       */
    SISPH_E_INVAL = -1,       /* invalid descriptor or argument              */
    SISPH_E_NOMEM = -2,       /* workspace or neighbour capacity too small   */
    SISPH_E_DEVICE = -3,      /* HIP runtime error                           */
    SISPH_E_STATE = -4,       /* call out of order                           */
    SISPH_E_NONFINITE = -5    /* NaN/Inf found by the PPE residual reduction */
};

/* ----------------------------------------------------------- enumerations */
enum { SISPH_QUINTIC = 0, SISPH_WENDLAND_C2 = 1 };      /* support 3h / 2h  */
enum { SISPH_FP64 = 0, SISPH_MIXED = 1, SISPH_FP32 = 2 }; /* see precision   */
enum { SISPH_ASYMM = 0, SISPH_SYMM = 1 };                /* pressure gradient */
enum { SISPH_GTVF_OFF = 0, SISPH_GTVF_INTERNAL = 1, SISPH_GTVF_EXTERNAL = 2 };
enum { SISPH_PREF_FIXED = 0, SISPH_PREF_TWICE_MAX = 1 };
enum { SISPH_CONV_SUM = 0, SISPH_CONV_MEAN = 1 };
enum { SISPH_USTAR_SLIP = 0, SISPH_USTAR_NOSLIP = 1 };
enum { SISPH_DT_FIXED = 0, SISPH_DT_ADAPTIVE = 1 };
enum { SISPH_JACOBI = 0, SISPH_BICGSTAB = 1 };
enum { SISPH_NULL_NONE = 0, SISPH_NULL_PROJECT = 1 };

/* One case.  Parameters follow the paper's statement of the problem.
 *  precision   SISPH_FP64: every sum in FP64.  SISPH_MIXED: neighbour sums,
 *              kernel values and the cached PPE coefficients in FP32 (pair
 *              differences formed in FP64 first); PPE residual, convergence
 *              test, per-particle results and positions in FP64.
 *              SISPH_FP32: plain single precision, the form the paper's own
 *              GPU runs use: as MIXED for the neighbour sums, and every
 *              per-particle result (density, accelerations, u*, r*, RHS,
 *              D_ii, the Jacobi update, the wall pressure, u^{n+1}, the GTVF
 *              sub-steps, the transport velocity, the positions) rounded to
 *              FP32 as it is formed, the PPE residual sums and the stopping
 *              test in FP32 too (arrays keep their FP64 storage, holding
 *              FP32 values).  Jacobi only.
 *  pgrad       "asymm" (eq. mom:sph:press:pij) or "symm" (eq. ...:symm).
 *  gtvf        OFF; INTERNAL: h~ = h, p0 = p_ref; EXTERNAL: h~ = h/2,
 *              p0 = min(10 |p_i|, p_ref) (section 2.1).
 *  free_surface  enables the rho/rho0 < fs_ratio flag (p = 0) and the
 *              clamp p_wall >= 0 (sections 3 and 3.4).
 *  p_ref_mode  FIXED: p_ref as given; TWICE_MAX: 2 max_i p_i after the first
 *              step's solve, then held.
 *  conv_norm   SUM: sum|dp| / max(Lambda, sum|p|) as printed; MEAN: Lambda
 *              scaled by the fluid count.
 *  forced_iters  > 0: run exactly that many sweeps (ignores tol).
 *  eta         the 0.01 of r^2 + eta h^2.
 *  dx          initial particle spacing; sizes the neighbour storage.
 *  nbr_cap     neighbour slots per particle (0: derived from h and dx).
 *  ustar_wall  wall ghost form for u* in the PPE: SISPH_USTAR_SLIP (the
 *              Shepard average of u*) or SISPH_USTAR_NOSLIP (2 u_wall minus
 *              it); either way any part into the solid is removed.
 *  dt_mode     SISPH_DT_FIXED: every step takes dt.  SISPH_DT_ADAPTIVE
 *              (section 3.2, adaptive steps): the first step takes dt; each
 *              later one min(dt, 0.25 h / max|u^n|, 0.25 sqrt(h / max|f^n|))
 *              from the previous step's largest fluid speed at its start
 *              and largest total acceleration (predictor forces, gravity
 *              and pressure force); dt is the upper bound.
 *  solver      SISPH_JACOBI: the paper's damped Jacobi sweeps (eq. p-sor).
 *              SISPH_BICGSTAB: BiCGStab (the alternative of section 3.1) on
 *              the same cached coefficients, scaled by D_ii; wall neighbours
 *              enter through the unclamped Shepard extrapolation (eq.
 *              p-shepard); stops when omega * sum|scaled residual| /
 *              max(Lambda, sum|p|) < tol (eq. convergence with the Jacobi
 *              update of the current iterate).  Free-surface problems only
 *              (without p = 0 rows the system fixes p only up to a
 *              constant); such a context cannot join a batch.  iters counts
 *              BiCGStab iterations (two operator applications each).
 *  null_space  SISPH_NULL_NONE: the iteration as printed.  SISPH_NULL_PROJECT
 *              (fully periodic cases only: no wall particles, no free
 *              surface, Jacobi): there a constant pressure solves the
 *              homogeneous PPE (every row of eq. sph-ppe sums c_ij (p_j -
 *              p_i)), y_i = m_i rho_i is a left null vector of the operator,
 *              and a right-hand side with y . RHS != 0 makes every sweep of
 *              eq. p-sor shift the iterate by the same constant, which the
 *              test of eq. convergence never sees settle.  Before the sweeps
 *              RHS_i becomes RHS_i - beta D_ii with beta = (y . RHS) /
 *              (y . D), and Lambda is taken from it; iterate k then equals
 *              the unprojected one minus k omega beta, the same field up to
 *              a constant.  Other cases are refused (SISPH_E_INVAL).
 *  periodic    per axis; the box is [box_lo, box_hi) on periodic axes and
 *              the binning range (particles outside are clamped to the edge
 *              cells) on the others.                                         */
typedef struct {
    int32_t dim, kernel, precision, pgrad, gtvf, free_surface;
    int32_t p_ref_mode, conv_norm, min_iter, max_iter, gtvf_K, forced_iters;
    int32_t periodic[3], nbr_cap;
    int32_t ustar_wall, dt_mode;
    int32_t solver, null_space;
    int64_t n_fluid, n_wall;
    double h, dx, rho0, nu, alpha, c_ref, dt, eta, fs_ratio, omega, tol, p_ref;
    double gravity[3], box_lo[3], box_hi[3];
} sisph_case_desc;

typedef struct {
    int32_t iters;       /* Jacobi sweeps done                              */
    int32_t converged;   /* final ratio < tol                               */
    int32_t nonfinite;   /* a non-finite pressure sum was seen              */
    int32_t status;      /* this case's status code (SISPH_OK, ...)      */
    double ratio;        /* eq. convergence at the last sweep               */
    double lambda;       /* max |RHS_i / D_ii| over non-free-surface fluid   */
    double p_ref;        /* GTVF reference pressure in use                  */
    double dt;           /* this step's time step                          */
    int32_t index_bits;  /* bits per neighbour index the sweeps read: 32
                            (the lists); 16 (offsets: mixed mode, no walls,
                            every offset of the step within +-32767); 12
                            (walled Jacobi cases on grids periodic in no
                            direction: the neighbour's position in the
                            workgroup's LDS copy of the iterate; the
                            workgroups whose copy would not fit read the
                            lists, list_blocks below)                      */
    int32_t list_blocks; /* packed mode: fluid workgroups (of 256 rows)
                            whose sweeps read the lists this step          */
    double beta;         /* SISPH_NULL_PROJECT: the constant removed per unit
                            D_ii from the RHS (else 0)                      */
} sisph_ppe_stats;

typedef sisph_ppe_stats sisph_step_stats;

typedef struct sisph_ctx sisph_ctx;

/* Exact device-workspace bytes a case needs (0 for an invalid descriptor). */
size_t sisph_workspace_bytes(const sisph_case_desc *desc);

/* Creates a context.  d_workspace: device memory of ws_bytes >=
 * sisph_workspace_bytes(desc), 256-byte aligned, owned by the caller and
 * kept alive until sisph_destroy.  x [n][dim], p [n], m [n] cover fluid and
 * walls; u [n_fluid][dim]; wall_u [n_wall][dim] is the prescribed (constant)
 * wall velocity or NULL for static walls.  Host arrays are copied; the
 * transport velocity starts equal to u.  hip_stream: the stream all work is
 * queued on (NULL: the default stream).  Wall normals are computed here. */
int32_t sisph_create(const sisph_case_desc *desc, void *d_workspace, size_t ws_bytes,
                     const double *x, const double *u, const double *p, const double *m,
                     const double *wall_u, void *hip_stream, sisph_ctx **out);

/* For callers that cannot allocate (code running under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): sisph_create with
 * the workspace taken from a library-owned device array of
 * SISPH_STATIC_WORKSPACE_BYTES per device (a static device variable, held
 * by every device the library runs on until the process ends) instead of
 * the caller's, on the current device.  It calls no hipMalloc, hipHostMalloc,
 * hipFree or hipEventCreate and allocates no host memory: the context and
 * its control-block mirror live in a static slot per device, and the
 * context has no timing events (its timings read zero; sisph_set_graphs,
 * sisph_set_kernel_timing and sisph_autotune refuse it with
 * SISPH_E_STATE).  Arguments as for sisph_create; hip_stream must belong
 * to the current device.  Errors: SISPH_E_NOMEM if the case needs more than
 * SISPH_STATIC_WORKSPACE_BYTES (sisph_workspace_bytes), SISPH_E_STATE while
 * a context created here on the same device is alive (one per device;
 * sisph_destroy releases it), SISPH_E_INVAL for a bad descriptor;
 * sisph_last_error(NULL) gives the message.  Every call on a device reuses
 * the same array, which keeps the previous case's contents; create sets up
 * every value a step reads.  Work of two threads on one device's static
 * context is not synchronised: such calls race. */
#define SISPH_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int32_t sisph_create_static(const sisph_case_desc *desc, const double *x, const double *u, const double *p,
                            const double *m, const double *wall_u, void *hip_stream, sisph_ctx **out);

int32_t sisph_bin(sisph_ctx *ctx);
int32_t sisph_predict(sisph_ctx *ctx);
int32_t sisph_ppe_solve(sisph_ctx *ctx, sisph_ppe_stats *out /* nullable */);
int32_t sisph_correct(sisph_ctx *ctx);
/* nsteps full steps; out: nsteps entries or NULL.  Returns the worst status
 * (errors stop the loop; SISPH_WARN_MAXITER does not). */
int32_t sisph_step(sisph_ctx *ctx, int32_t nsteps, sisph_step_stats *out);

/* State in the caller's original order: x [n][dim] (fluid then walls),
 * u and u_tilde [n_fluid][dim], p [n] (fluid then walls), rho [n_fluid].
 * Any pointer may be NULL.  Valid between steps. */
int32_t sisph_read_state(sisph_ctx *ctx, double *x, double *u, double *u_tilde,
                         double *p, double *rho);
/* Replaces the fluid state between steps (same layouts; NULL keeps). */
int32_t sisph_write_state(sisph_ctx *ctx, const double *x, const double *u,
                          const double *u_tilde, const double *p);

/* Diagnostic fields of the last step in original order (tests, reports). */
enum {
    SISPH_FIELD_RHO = 0,      /* [n_fluid]        at r^n                   */
    SISPH_FIELD_XSTAR = 1,    /* [n_fluid][dim]   r*                       */
    SISPH_FIELD_USTAR = 2,    /* [n_fluid][dim]   u*                       */
    SISPH_FIELD_RHS = 3,      /* [n_fluid]                                 */
    SISPH_FIELD_DII = 4,      /* [n_fluid]                                 */
    SISPH_FIELD_UNEW = 5,     /* [n_fluid][dim]   u^{n+1}                  */
    SISPH_FIELD_WALL_U = 6,   /* [n_wall][dim]    stage-1 ghost velocity   */
    SISPH_FIELD_WALL_USTAR = 7, /* [n_wall][dim]  stage-2 ghost u*         */
    SISPH_FIELD_FS = 8,       /* [n_fluid]        free-surface flag (0/1)  */
    SISPH_FIELD_NORMAL = 9,   /* [n_wall][dim]    wall unit normals        */
    SISPH_FIELD_PRESSURE = 10 /* [n]              current pressure         */
};
int32_t sisph_read_field(sisph_ctx *ctx, int32_t field, double *out);

/* Total number of stored neighbour pairs (self included) of the lists held
 * for stage / dest (as below); only the per-row counts leave the device. */
int32_t sisph_pair_count(sisph_ctx *ctx, int32_t stage, int32_t dest, int64_t *pairs);

/* Number of rows of those lists holding at least one particle other than
 * the row itself (wall rows without fluid neighbours are not read by any
 * sweep).  Same stage / dest as sisph_pair_count; only per-row counts leave
 * the device. */
int32_t sisph_rows_with_neighbours(sisph_ctx *ctx, int32_t stage, int32_t dest, int64_t *rows);

/* Neighbour sets as CSR in original ids, each row ascending.
 * stage 0: N^n (valid after sisph_bin), stage 1: N* (after sisph_predict);
 * dest 0: fluid rows over fluid+wall sources, dest 1: wall rows over fluid
 * sources.  offsets [rows+1]; ids up to cap entries. */
int32_t sisph_debug_neighbors(sisph_ctx *ctx, int32_t stage, int32_t dest,
                              int64_t *offsets, int32_t *ids, int64_t cap);

/* Wall-clock of the last sisph_ppe_solve measured with HIP events on the
 * context's stream, and of the whole last step (milliseconds). */
int32_t sisph_last_timings(sisph_ctx *ctx, double *ppe_ms, double *step_ms);

/* Accumulated since the last reset: HIP-event time of the Jacobi sweep
 * chunks (each chunk = sweeps queued back to back, with the wall-pressure
 * kernel of each sweep when the case has walls; for a persistent solve, its
 * one launch), the number of sweeps run (per-launch: one per launch), and
 * the number of those that advanced the solve (the rest found it already
 * finished).  reset != 0 clears after reading. */
int32_t sisph_sweep_counters(sisph_ctx *ctx, double *sweep_ms, int64_t *launches,
                             int64_t *effective, int32_t reset);

/* Timing of the Jacobi sweep kernel alone.  With period > 0 every
 * period-th sweep launch of each solve of a single context (launches 0,
 * period, 2 period, ... of the solve; 1: every launch) is bracketed by its
 * own pair of HIP events on the context's stream (the wall pressure pass
 * before it is left out; a persistent solve's one launch is timed whole),
 * from a pool of 2 (max_iter + 1) events created here; period <= 0 frees
 * the pool.  Off by default.  An event pair costs the stream a few
 * microseconds, so sampling keeps the timed run's pace.
 * sisph_kernel_timing returns, accumulated since the last reset of
 * sisph_sweep_counters, the summed kernel time of the timed launches in
 * milliseconds, their number (launches past a solve's stop included) and
 * how many of them were persistent solves.  Any pointer may be NULL. */
int32_t sisph_set_kernel_timing(sisph_ctx *ctx, int32_t period);
int32_t sisph_kernel_timing(sisph_ctx *ctx, double *ms, int64_t *launches, int64_t *persistent);

/* Persistent solves (see sisph_set_persistent) since the last counter reset
 * (kernel launches, one per solve), and whether the last solve was one. */
int32_t sisph_persistent_info(sisph_ctx *ctx, int64_t *solves, int32_t *last);

/* Since the last reset of sisph_sweep_counters, how often a solve meant
 * for one persistent launch ran as per-launch sweeps instead: the runtime refused the cooperative launch
 * (it is tried again on later solves; after eight refusals that first-batch
 * size is given up), or a workgroup waited
 * longer than the spin limit at a grid barrier (the solve was redone from
 * its starting iterate; the context keeps per-launch sweeps). */
int32_t sisph_persistent_fallbacks(sisph_ctx *ctx, int64_t *refused, int64_t *timed_out);

/* Graph replay of the fixed parts of a step (the data-dependent PPE loop
 * stays a sequence of polled launch chunks with device-side early exit):
 * with on != 0, sisph_step captures once, then replays, two HIP graphs per
 * context, the kernels from binning to the PPE set-up and those from the
 * settle of the pressure to the advance; results are bitwise those of the
 * launches one by one.  The stage calls (sisph_bin, ...) always launch
 * directly.  Off by default. */
int32_t sisph_set_graphs(sisph_ctx *ctx, int32_t on);

/* Single Jacobi solves of cases without walls whose fluid workgroups all fit
 * on the device at once run as one cooperative launch that holds every
 * sweep (on by default): the rows' coefficients stay in registers, the
 * workgroups meet at a grid barrier between sweeps and the host waits once
 * per solve instead of polling between chunks of launches.  Results and
 * sweep counts are bitwise those of the per-launch sweeps.  on = 0 keeps
 * the per-launch sweeps (used to compare the two).  The launch needs the
 * device's compute units to itself: a persistent solve of another context
 * running at the same time on the same device can keep a workgroup from
 * starting.  Every wait in the launch is bounded; when a barrier does not
 * fill in time the solve is redone from its starting iterate with
 * per-launch sweeps (same results), and the context keeps those from then
 * on.  Contexts solved concurrently on one device should turn the mode off
 * (each timeout costs a fraction of a second). */
int32_t sisph_set_persistent(sisph_ctx *ctx, int32_t on);

/* Test hook: the number of polls after which a wait of the persistent
 * solve gives up (0: at once, which exercises the fallback above). */
int32_t sisph_debug_barrier_spins(sisph_ctx *ctx, uint32_t spins);

/* Test hook: on = 0 makes a single context's sweeps read the neighbour
 * lists instead of the packed mode's LDS copy and codes (walled Jacobi
 * cases on grids periodic in no direction), on = 1 restores them; the sums
 * and their order are the same either way.  SISPH_E_INVAL for on = 1 on a
 * case without the packed mode. */
int32_t sisph_debug_packed(sisph_ctx *ctx, int32_t on);

/* Test hook.  With the external-flow GTVF (section 2.1: smoothing length
 * h/2, so the sub-steps of eq. mom:sph:gtvf reach only the closer part of
 * the neighbours) the neighbour build at r* also lists, per row, the
 * neighbours closer than the GTVF support plus a margin, and the sub-steps
 * walk that short list while no particle has moved more than 0.05 dx from
 * r*; a neighbour it leaves out adds exactly zero, so the sums are the same
 * bit for bit.  on = 0 makes the sub-steps walk the full lists, on = 1
 * restores the short lists, on = -1 changes nothing.  *used (host,
 * nullable) receives, for the last completed step, 0 if the case has no
 * short lists (or they are off), 1 if every sub-step walked them, 2 if one
 * walked the full lists (a short list overflowed, or a particle moved past
 * the bound).  SISPH_E_INVAL for on = 1 on a case without them,
 * SISPH_E_STATE while attached to a batch. */
int32_t sisph_debug_gtvf_short(sisph_ctx *ctx, int32_t on, int32_t *used);

/* Measurement aid, not part of the method: the device's plain read rate,
 * the ceiling of a kernel that streams its operands once.  Reads the first
 * `bytes` (a positive multiple of 16) of the device buffer `buf` `reps`
 * times with a grid-stride kernel of 16-byte loads, `grid` workgroups of 256
 * threads, each thread writing one float into `out` (device, grid * 256
 * floats), on the null stream after the work queued there, and stores the
 * average time of one read in microseconds (HIP events) in *us (host).
 * Both buffers are the caller's.  SISPH_E_INVAL for a null pointer or a bad
 * size, grid or reps; SISPH_E_DEVICE on a HIP error. */
int32_t sisph_debug_read_rate(const void *buf, int64_t bytes, float *out, int32_t grid, int32_t reps,
                              double *us);

int32_t sisph_destroy(sisph_ctx *ctx);

/* ------------------------------------------------------------- autotuning
 * The Jacobi sweep comes in SISPH_SWEEP_VARIANTS launch variants (how many
 * neighbour slots are fetched in the first round trip, and whether
 * workgroups are mapped to XCDs in contiguous ranges).  They differ in speed
 * only: every variant computes the same sums in the same order.
 * sisph_autotune times each variant `reps` times on the context's current
 * state (it needs one completed step; it writes only the scratch iterate, so
 * the simulation state is unchanged), selects the fastest and returns it in
 * *best and the mean launch time of every variant in us[] (microseconds,
 * SISPH_SWEEP_VARIANTS entries, nullable).  A batch launches its group with
 * the variant of its largest case. */
enum { SISPH_SWEEP_VARIANTS = 8 };
int32_t sisph_autotune(sisph_ctx *ctx, int32_t reps, int32_t *best, double *us);
int32_t sisph_set_variant(sisph_ctx *ctx, int32_t variant);
int32_t sisph_get_variant(sisph_ctx *ctx);

/* ------------------------------------------------------------- batching
 * Many independent cases stepped together: every kernel of a step is one
 * launch over all attached cases that share dimension, kernel and
 * precision (each workgroup finds its case in a device table), and each
 * case keeps its own PPE convergence (a converged case's sweeps return at
 * once).  A case gives the same results alone and in a batch, bit for bit:
 * its workgroups, sums and decisions do not depend on the other cases.
 * The batch owns small device tables (allocated here, freed by
 * sisph_batch_destroy); the cases' workspaces stay with their callers.
 * Attached contexts must be between steps and on the batch's stream; while
 * attached they are stepped only through the batch.  Not thread-safe. */
typedef struct sisph_batch sisph_batch;

int32_t sisph_batch_create(int32_t max_cases, void *hip_stream, sisph_batch **out);
int32_t sisph_batch_attach(sisph_batch *b, sisph_ctx *ctx);
int32_t sisph_batch_detach(sisph_batch *b, sisph_ctx *ctx);
int32_t sisph_batch_size(sisph_batch *b);
/* One SISPH step of every attached case.  per_case: sisph_batch_size(b)
 * entries in attach order (or NULL).  Returns the worst status over the
 * cases (errors of single cases are reported in their entries' nonfinite
 * flag and in the return value). */
int32_t sisph_batch_step(sisph_batch *b, sisph_step_stats *per_case);
/* As sisph_set_graphs, per (dimension, kernel, precision) group of the batch;
 * graphs are captured again after the group's membership changes. */
int32_t sisph_batch_set_graphs(sisph_batch *b, int32_t on);
/* Jacobi solves of the wall-less cases of a (dimension, kernel, precision)
 * group in one cooperative launch (on by default) when all their fluid
 * workgroups fit on the device at once: each case keeps its own stopping
 * decision and results bitwise those of per-launch sweeps; the group's
 * cases with walls then take per-launch sweeps.  A refused launch or a grid
 * barrier that does not fill in time falls back to per-launch sweeps for
 * that step.  sisph_batch_persistent_info counts, since the batch's
 * creation, such launches and the fallbacks. */
int32_t sisph_batch_set_persistent(sisph_batch *b, int32_t on);
int32_t sisph_batch_persistent_info(sisph_batch *b, int64_t *launches, int64_t *fallbacks);
int32_t sisph_batch_destroy(sisph_batch *b);

const char *sisph_status_string(int32_t status);
/* Last error message of this context (or of the last failed create). */
const char *sisph_last_error(sisph_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
