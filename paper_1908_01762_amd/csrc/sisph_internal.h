// Internal types of libsisph: device-side parameter blocks, the per-case
// state (pointers carved out of the caller's workspace) and the launch
// interface the host runtime uses.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sisph.h"

namespace sisph {

constexpr int kBlock = 256;   // threads per workgroup for particle kernels

// FP32 neighbour sums and FP32 copies of gathered fields: the mixed mode and
// the plain FP32 mode.
__host__ __device__ inline bool f32_sums(int precision) { return precision != SISPH_FP64; }
constexpr int kXcd = 8;       // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

// Binning grid and periodic box.  Cell edge >= R (with a 1e-6 margin), so
// two particles closer than R are never more than one cell apart.
struct Grid {
    double lo[3], hi[3], L[3], Lh[3];
    double edge[3];
    int32_t nc[3];
    int32_t per[3];
    int64_t ncell;
};

// Scalar parameters of one case as kernels see them.
struct Params {
    int32_t dim, kernel, precision, pgrad, gtvf, free_surface;
    int32_t conv_norm, min_iter, max_iter, forced_iters, gtvf_K, cap;
    int32_t ustar_noslip;   // wall ghost form for u*: 0 slip, 1 no-slip
    int32_t adaptive_dt;    // next dt from this step's maxima
    int32_t solver;         // SISPH_JACOBI or SISPH_BICGSTAB
    int32_t compact;        // mixed mode without walls: 16-bit neighbour offsets
    int32_t packed;         // walled Jacobi cases not periodic in x: 12-bit neighbour codes
                            // (positions in the workgroup's LDS copy of the iterate)
    // External-flow GTVF (smoothing length h/2, so the sub-steps reach only
    // part of the neighbours): the sub-steps walk a short list built with
    // the r* lists, of the neighbours closer than sqrt(g_R2); it holds
    // while no particle has moved more than sqrt(g_D2) from r*
    int32_t g_sub, g_cap;
    double g_R2, g_D2;
    // every particle has the same mass (m_uni_f: it in FP32): the FP32-sum
    // predictor's neighbour record then leaves it out (64 bytes, not 80)
    int32_t m_uni;
    float m_uni_f;
    uint32_t barrier_spins; // polls before a wait of the persistent solve gives up
    int32_t null_space;     // SISPH_NULL_PROJECT: RHS made compatible before the sweeps
    int64_t nf, nw, ntot;
    // dt: the fixed step, or the first step and the upper bound when adaptive
    // (kernels read the current step's dt from Control)
    double h, rho0, nu, alpha, c_ref, dt, eps_h, fs_ratio, omega, tol;
    double R2;      // (support * h)^2, the exact neighbour predicate radius^2
    double g[3];
    Grid grid;
};

// Device control block of one case: PPE loop state and reduction results.
struct Control {
    int32_t iter;          // sweeps done in the current solve
    int32_t done;          // solve finished (converged, max_iter, forced)
    int32_t stopped_at;    // sweep count at which the solve stopped (INT32_MAX: running)
    int32_t nonfinite;     // a non-finite pressure sum was seen
    int32_t overflow;      // neighbour capacity exceeded
    int32_t maxcnt;        // largest neighbour count seen (on overflow)
    int32_t p_ref_set;
    int32_t barrier_late;  // a grid barrier of the persistent solve timed out
    double ratio, num, den;
    unsigned long long lambda_bits;   // max |RHS/D| (non-negative doubles)
    unsigned long long pmax_key;      // max p, order-preserving key
    double p_ref;
    double dt;                        // this step's time step
    double dt_next;                   // the next step's (taken at its start)
    unsigned long long umax2_bits;    // max |u^n|^2 over fluid (adaptive dt)
    unsigned long long fmax2_bits;    // max |f^n|^2 over fluid (adaptive dt)
    // BiCGStab scalars of iterations k (slot k & 1): rho_k = (r^, r_{k-1}),
    // alpha_k, omega_k; a zero step denominator sets brk
    double bicg_rho[2], bicg_alpha[2], bicg_omega[2];
    int32_t bicg_brk;
    int32_t wide;                     // a neighbour offset of this step did not fit 16 bits
    int32_t pk_overflow;              // packed mode: workgroups of this step that read the lists
    int32_t g_full;                   // the GTVF short list overflowed this step
    unsigned long long g_disp_bits;   // max |r^k - r*|^2 over the GTVF sub-steps so far
    double beta;                      // SISPH_NULL_PROJECT: (y . RHS) / (y . D), y = m rho
};

// Per-case device arrays.  Unified particle index: fluid [0, nf) in cell
// order (re-sorted every step), walls [nf, nf + nw) in static cell order.
struct State {
    double *x[3];      // r^n                        [ntot]
    double *u[3];      // u^n fluid, wall ghost u    [ntot]
    double *ut[3];     // transport velocity         [nf]
    double *xs[3];     // r*                         [ntot]
    double *us[3];     // u* fluid, wall slip u*     [ntot]
    double *un[3];     // u^{n+1}                    [nf]
    // GTVF sub-step records {x, y, z, m/rho^2}: one 32-byte gather per
    // neighbour; the seed (r*) in gk[1], sub-step k writes gk[k & 1]
    double4 *gk[2];    // [ntot] x2
    int32_t *gnbr, *gcnt;   // GTVF short lists (g_sub): [g_cap][nf], [nf]
    double *vk[3];     // GTVF sub-step velocity     [nf]; before the sub-steps,
                       // the step's total acceleration (adaptive dt)
    double *nrm[3];    // wall unit normals          [nw]
    double *wallu[3];  // prescribed wall velocity   [nw]
    double *p[2];      // pressure iterates; p[0] holds p^n between steps [ntot] x2
    float *p32;        // FP32 copies of the iterates (mixed) [2][ntot]
    double *m;         // mass                       [ntot]
    double *rho;       // density (walls rho0)       [ntot]
    void *mr2;         // m / rho^2 in the working precision [ntot]
    // FP32 copies for the mixed-mode pair gathers (see Shadow)
    float *m32, *rho32;        // [ntot]
    // the gathered fields of the predictor, the PPE coefficients or the
    // pressure force, one record per particle (PredRec, CoefRec, CorrRec)
    void *prec;                // [ntot]
    double *rhs, *dii; //                            [nf]
    int32_t *fs;       // free-surface flag          [nf]
    int32_t *id;       // original index of sorted fluid slot [nf]
    int32_t *wid;      // original wall index of sorted wall slot [nw]
    // binning
    uint32_t *key, *rank, *count, *fstart, *wstart, *scan_tmp;
    int32_t *perm;          // sorted slot -> source index (at r*: cell slot -> particle)
    // neighbour lists, slot-major [cap][n]: slot 0 is the particle itself
    int32_t *nbr, *cnt;     // fluid rows: fluid + wall sources
    int32_t *wnbr, *wcnt;   // wall rows: fluid sources
    void *coef;             // cached PPE c_ij, working precision, group-major [cap/4][nf][4]
    void *cidx;             // their indices (int32) or 16-bit offsets (compact) or codes (packed), same layout
    // packed mode: eight 12-bit staged positions per 12-byte word,
    // group-major [ceil((cap - 1) / 8)][nf] (word w of a row holds list
    // slots 8w + 1 .. 8w + 8), and per fluid workgroup its staging record
    uint3 *pk12;
    int32_t *stagerec;      // [nblk][kStageRec]
    // packed mode with FP32 sums: the row words the sweep reads, RHS and
    // D_ii (FP32 sums, so their FP32 values are exact) and the neighbour
    // count with the free-surface flag in bit 31                     [nf]
    float2 *rd32;
    int32_t *cf;
    void *wcoef;            // cached wall weights W_wf / sum W: FP32 sums: (f, weight) words, each
                            // row's run at woffw[w]; FP64: weights [cap][nw] (indices from wnbr)
    double *wh;             // wall hydrostatic term                 [nw]
    int32_t *wflag;         // wall workgroup has a row with fluid neighbours at r*   [nwb]
    int32_t *wblk;          // [0] = count, then those workgroups in order            [1 + nwb]
    uint32_t *wsum;         // per wall workgroup: rows with fluid neighbours, their entries;
                            // then exclusive prefixes; [2 nwb] = totals                 [2 nwb + 2]
    uint2 *wrow;            // rows with fluid neighbours in wall order: (w, first word);
                            // [rows] = (~0, all words)                                    [nw + 1]
    uint32_t *woffw;        // each wall row's first word                                 [nw]
    double *partial;        // per-workgroup partial sums of two sweeps [2][2][nblk]
    double *tmp;            // reorder scratch [16][max(nf, nw)]
    // BiCGStab (solver only): x, r, r^, p, v, s, t, scaled RHS f, wall
    // hydrostatic part h, each [ntot] (wall slots of x, p, s hold their
    // extrapolation), and six partial-sum rows [6][nblk]
    double *bx, *br, *brh, *bp, *bv, *bs, *bt, *bf, *bh, *bpart;
    Control *ctl;
    // Persistent solve, apart from the Control fields written with ordinary
    // stores: [0] a barrier timed out; at kSyncBcast + 64 x (x < kSyncCopies,
    // one 256-byte line each) the word workgroup 0 posts after each sweep;
    // at kSyncArrive + b the sweeps workgroup b has finished
    uint32_t *sync;
};

// The fields the predictor gathers for a neighbour, in one record (five or
// six 16-byte loads instead of eleven scattered ones): r^n, u^n (walls:
// the ghost velocity), the transport velocity (fluid; 0 for walls), mass and
// density in the working precision.
struct __align__(16) PredRecF {
    double x[3], u[3], ut[3];
    float m, rho;
};
struct __align__(16) PredRecD {
    double x[3], u[3], ut[3];
    double m, rho;
};
// The FP32-sum record when every particle has the same mass: r^n and u^n in
// FP64, u~ - u formed in FP64 and rounded to FP32 (as the pair term did; 0
// for walls), density in FP32: 64 bytes, four loads instead of five.
struct __align__(16) PredRecS {
    double x[3], u[3];
    float s[3], rho;
};
// The same for the PPE coefficients (r*, u* (walls: the slip ghost), mass
// and density) and for the pressure force (r*, the solved pressure,
// density in FP64 and mass in the working precision), written into the same
// buffer before each of them.
struct __align__(16) CoefRecF {
    double x[3], u[3];
    float m, rho;
};
struct __align__(16) CoefRecD {
    double x[3], u[3];
    double m, rho;
};
struct __align__(16) CorrRec {
    double x[3], p, rho, m;
};
// The symmetric form in FP32 sums needs of a neighbour only r*, m and
// p / rho^2 (formed in FP64, rounded to FP32, as the pair term would):
// 32 bytes, two loads.
struct __align__(16) CorrRecS {
    double x[3];
    float q, m;
};

// Launch-size kinds: how many workgroups one case needs for a kernel.
constexpr int kWallRunBlocks = 2048;   // grid of the per-sweep wall pass (K_WALLRUN launches)
constexpr int kCellsPerWave = 2;   // cells one wavefront sorts, one per 32 lanes (K_CELLW launches)

enum Kind { K_FLUID = 0, K_WALL, K_TOT, K_CELL, K_TILE, K_ONE, K_CELLW, K_WALLRUN, K_COUNT };

// Packed mode (walled Jacobi cases on grids periodic in no direction):
// each sweep workgroup copies the iterate of the particles its rows can
// reach into LDS, at most kStageBytes of values, and a neighbour is stored
// as its 12-bit position in that copy.  The copy is 2 NR index intervals
// (NR = 3^(D-1) stencil rows, fluid then walls); a workgroup's record holds
// whether it is staged, each interval's first global index and the
// intervals' positions in the copy (prefix sums): kStageRec words.
constexpr int kStageBytes = 16384;
constexpr int kStageRec = 40;

__host__ __device__ inline int64_t kind_blocks(const Params &P, int kind) {
    switch (kind) {
    case K_FLUID: return (P.nf + kBlock - 1) / kBlock;
    case K_WALL: return (P.nw + kBlock - 1) / kBlock;
    case K_TOT: return (P.ntot + kBlock - 1) / kBlock;
    case K_CELL: return (P.grid.ncell + kBlock - 1) / kBlock;
    case K_TILE: return (P.grid.ncell + kScanTile - 1) / kScanTile;
    case K_WALLRUN: {   // the per-sweep wall pass: a grid-stride loop over the compact rows
        const int64_t nb = (P.nw + kBlock - 1) / kBlock;
        return nb < kWallRunBlocks ? nb : kWallRunBlocks;
    }
    case K_CELLW: return (P.grid.ncell + kBlock / 64 * kCellsPerWave - 1) / (kBlock / 64 * kCellsPerWave);
    default: return 1;
    }
}

// One case of a batch as the batched kernels see it.
struct CaseEntry {
    Params P;
    State S;
    int64_t nblk[K_COUNT];
};

// Where a group of launches goes: one case (parameters by value) or a batch
// of cases of the same dimension, kernel and precision (a device table; a
// per-kind map from workgroup to case and the case's first workgroup).
struct Target {
    const Params *P;
    const State *S;
    const CaseEntry *tab;            // device
    const int32_t *owner[K_COUNT];   // device: case of each workgroup
    const int64_t *first[K_COUNT];   // device: first workgroup of each case
    int64_t total[K_COUNT];          // workgroups per kind over the batch
    int32_t ncase;
    int32_t dim, kernel, precision;
    int32_t variant;                 // Jacobi-sweep variant (speed only)
    int32_t adaptive;                // some case chooses its next dt
    int32_t packed;                  // some case stores packed neighbour codes
    // the sweep tests the stop flag before its other loads: batches (cases
    // stop at different counts) and large cases (a launch beyond the stop
    // would read every row), see precheck_for()
    int32_t precheck;
    int32_t solver;                  // SISPH_JACOBI or SISPH_BICGSTAB (single cases)
    int32_t null_space;              // some case projects its RHS (SISPH_NULL_PROJECT)
    bool batched;
    hipStream_t s;
};

// RESET_DT: dt = dt_next = the case's dt (at creation); RESET_STEP: start a
// step (dt = dt_next, maxima cleared).
enum { RESET_PPE = 1, RESET_NEIGHBOURS = 2, RESET_PREF = 4, RESET_DT = 8, RESET_STEP = 16 };
enum { POS_X = 0, POS_XS = 1 };

// ---- launch sequences (sisph_kernels.hip) -------------------------------
void reset_control(const Target &T, int what);
// Stable counting sort of the fluid at r^n (POS_X, data reordered into cell
// order) or at r* (POS_XS, cell slots map through perm).
void bin_fluid(const Target &T, int which);
// Walls of a single case, once at creation.
void bin_walls_once(const Target &T);
// Neighbour lists at r^n (POS_X; with them the summation density and
// free-surface flag) or at r* (POS_XS; then the packed codes).
void build_neighbors(const Target &T, int which);
void wall_normals(const Target &T);
void mass_over_rho2(const Target &T);
// FP32 copies of mass and density (mixed mode), after the density.
void shadow(const Target &T);
// Wall ghost velocity: no-slip form at r^n (POS_X); at r* (POS_XS) the
// case's form for u* (slip by default).
void wall_velocity(const Target &T, int which);
void predictor(const Target &T);
void rhs_coef(const Target &T);
// SISPH_NULL_PROJECT cases: beta from the per-workgroup sums rhs_coef left,
// then RHS_i -= beta D_ii and Lambda from the result.
void project_rhs(const Target &T);
// Wall extrapolation weights at r* for the solve (walls present).
void wall_coef(const Target &T);
void copy_p32(const Target &T);
// Jacobi: wall pressure and sweep L.  BiCGStab: iteration L+1 (its first
// kernel decides whether the solve stopped after L iterations).
void ppe_iteration(const Target &T, int launch);
// BiCGStab set-up (x = p^n, r = f - M x, r^ = r) and final copy of x into p[0].
void bicg_begin(const Target &T);
void bicg_settle(const Target &T);
// The sweep alone (no wall pressure), for timing variants; the wall
// pressure pass of Jacobi sweep L alone.
void sweep_only(const Target &T, int launch);
void wall_pressure_iteration(const Target &T, int launch);
// Fluid rows from which a single case's sweep tests the stop flag first.
constexpr int64_t kPrecheckRows = int64_t(1) << 19;
// Sweep launch variants: kSweepFirstCount first-batch sizes, each with
// XCD-contiguous (v < kSweepFirstCount) or hardware workgroup order.
constexpr int kSweepFirstCount = 4;
constexpr int kSweepVariants = 2 * kSweepFirstCount;
constexpr int kDefaultVariant = 2;   // 20 neighbours first, XCD-contiguous
void settle_pressure(const Target &T);
// The whole Jacobi solve of one wall-less case in one cooperative launch
// (every workgroup resident); returns the launch's error.  The capacity is
// the number of fluid workgroups such a launch can hold (0: none).
hipError_t ppe_persistent(const Target &T, int limit);
int64_t ppe_persistent_capacity(const Target &T);
constexpr uint32_t kBarrierSpins = 1u << 18;   // polls before a grid barrier gives up
constexpr int kSyncCopies = 8;                 // one posted word per XCD
constexpr int kSyncBcast = 64, kSyncArrive = 64 * (1 + kSyncCopies);
constexpr int kSyncWords = kSyncArrive + 1024;   // at most 1024 workgroups
// The Jacobi solves of a batch's wall-less cases in one cooperative launch:
// ptotal workgroups, powner / pfirst mapping each to its case (index into
// the batch table) and to the case's first workgroup; bsync holds the
// barrier words, the cases stopped so far and per-case stop words (see
// kBatchSyncWords), prepared by the caller.
hipError_t ppe_persistent_batch(const Target &T, const int32_t *powner, const int64_t *pfirst, int64_t ptotal,
                                uint32_t *bsync, int ncase, int limit, uint32_t spins);
int64_t ppe_persistent_batch_capacity(const Target &T);
// bsync layout: [0] late flag, [32] cases stopped, [kSyncBcast + 64 x]
// posted words, [kSyncArrive + b] arrivals, [kSyncArrive + 1024 + c] case c's
// stop (0xffffffff: running)
constexpr int64_t kBatchSyncStop = kSyncArrive + 1024;
inline int64_t batch_sync_words(int64_t ncase) { return kBatchSyncStop + ncase; }
void wall_pressure_final(const Target &T);
void pressure_max(const Target &T);
void correct(const Target &T);
// Adaptive dt: max |u^n|^2 and max |f^n|^2 over the fluid, then dt_next.
void step_maxima(const Target &T);
void next_dt(const Target &T);
void gtvf_substep(const Target &T, int k);
void advance(const Target &T);
void gtvf_seed(const Target &T);
void coef_seed(const Target &T);
void corr_seed(const Target &T);
void gather_control(const Target &T, Control *out);

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_f64(double *p, double v, int64_t n, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);
// The plain FP32 mode's starting state rounded to FP32 (nothing otherwise).
void round_state(const Target &T);
// Row-major [n][dim] device array -> the SoA component arrays dst[k] + at.
void aos_to_soa(const double *src, double *const dst[3], int64_t at, int dim, int64_t n, hipStream_t s);

}  // namespace sisph
