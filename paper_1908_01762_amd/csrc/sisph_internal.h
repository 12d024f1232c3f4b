// Internal types of libsisph: device-side parameter blocks, the per-case
// state (pointers carved out of the caller's workspace) and the launchers the
// host runtime calls.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sisph.h"

namespace sisph {

constexpr int kBlock = 256;   // threads per workgroup for particle kernels
constexpr int kXcd = 8;       // MI355X: 8 XCDs, workgroups dealt round-robin

// Binning grid and periodic box.  Cell edge >= R (with a 1e-6 margin), so
// two particles closer than R are never more than one cell apart.
struct Grid {
    double lo[3], hi[3], L[3], Lh[3];
    double edge[3];
    int32_t nc[3];
    int32_t per[3];
    int64_t ncell;
};

// Scalar parameters of one case as kernels see them (passed by value).
struct Params {
    int32_t dim, kernel, precision, pgrad, gtvf, free_surface;
    int32_t conv_norm, min_iter, max_iter, forced_iters, gtvf_K, cap;
    int64_t nf, nw, ntot;
    double h, rho0, nu, alpha, c_ref, dt, eps_h, fs_ratio, omega, tol;
    double R2;      // (support * h)^2, the exact neighbour predicate radius^2
    double g[3];
    Grid grid;
};

// Device control block of one case: PPE loop state and reduction results.
struct Control {
    int32_t iter;          // sweeps done in the current solve
    int32_t done;          // solve finished (converged, max_iter, forced)
    int32_t nonfinite;     // a non-finite pressure sum was seen
    int32_t overflow;      // neighbour capacity exceeded
    int32_t maxcnt;        // largest neighbour count seen
    uint32_t ticket;       // last-workgroup-done counter
    int32_t p_ref_set;
    int32_t pad;
    double ratio, num, den;
    unsigned long long lambda_bits;   // max |RHS/D| (non-negative doubles)
    unsigned long long pmax_key;      // max p, order-preserving key
    double p_ref;
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
    double *xk[2][3];  // GTVF sub-step positions    [ntot] x2
    double *vk[3];     // GTVF sub-step velocity     [nf]
    double *nrm[3];    // wall unit normals          [nw]
    double *wallu[3];  // prescribed wall velocity   [nw]
    double *p[2];      // pressure iterates          [ntot] x2
    float *p32;        // FP32 copy of the current iterate (mixed) [ntot]
    double *m;         // mass                       [ntot]
    double *rho;       // density (walls rho0)       [ntot]
    double *rhs, *dii; //                            [nf]
    int32_t *fs;       // free-surface flag          [nf]
    int32_t *id;       // original index of sorted fluid slot [nf]
    int32_t *wid;      // original wall index of sorted wall slot [nw]
    // binning
    uint32_t *key, *rank, *count, *fstart, *wstart, *scan_tmp;
    int32_t *perm, *items;
    // neighbour lists, slot-major [cap][n]: slot 0 is the particle itself
    int32_t *nbr, *cnt;     // fluid rows: fluid + wall sources
    int32_t *wnbr, *wcnt;   // wall rows: fluid sources
    void *coef;             // cached PPE c_ij, float (mixed) or double [cap][nf]
    double *partial;        // per-workgroup partial sums, two sweeps [2][2][nblk]
    double *tmp;            // reorder scratch [ntot]
    Control *ctl;
    int64_t nblk_f;         // workgroups of a fluid launch
};

// ---- launchers (sisph_kernels.hip) -------------------------------------
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_f64(double *p, double v, int64_t n, hipStream_t s);
enum { RESET_PPE = 1, RESET_NEIGHBOURS = 2, RESET_PREF = 4 };
void reset_control(Control *c, int what, hipStream_t s);

// Stable counting sort of [base, base+n) by cell of pos; perm gets, per
// sorted slot, the source index (relative to base).  sortkey (nullable)
// orders particles within a cell (otherwise the source index does).
void bin_particles(const Params &P, const double *const pos[3], int64_t base, int64_t n,
                   const int32_t *sortkey, State &S, uint32_t *start, int32_t *perm,
                   hipStream_t s);
void reorder_f64(const int32_t *perm, int64_t n, double *const *arrays, int narr,
                 double *tmp, hipStream_t s);
void reorder_i32(const int32_t *perm, int64_t n, int32_t *a, int32_t *tmp, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);

void build_neighbors(const Params &P, const double *const pos[3], State &S, hipStream_t s);

void wall_normals(const Params &P, State &S, hipStream_t s);
void density(const Params &P, State &S, hipStream_t s);
void wall_velocity(const Params &P, const double *const pos[3], const double *const uf[3],
                   double *const uw[3], int slip, State &S, hipStream_t s);
void predictor(const Params &P, State &S, hipStream_t s);
void rhs_coef(const Params &P, State &S, hipStream_t s);
void ppe_iteration(const Params &P, State &S, int launch, hipStream_t s);
void wall_pressure_final(const Params &P, State &S, hipStream_t s);
void pressure_max(const Params &P, State &S, int final_parity, hipStream_t s);
void correct(const Params &P, State &S, int final_parity, hipStream_t s);
void gtvf_substep(const Params &P, State &S, int final_parity, int k, hipStream_t s);
void advance(const Params &P, State &S, int kfinal, hipStream_t s);
void copy_p32(const Params &P, State &S, hipStream_t s);

}  // namespace sisph
