/* SISPH oracle: a plain, serial, FP64 CPU implementation of one time step of
 * the simple iterative ISPH scheme (Muta, Ramachandran & Negi, "An efficient,
 * open source, iterative ISPH scheme", arXiv:1908.01762).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the HIP path.
 *
 * Conventions: arrays are row-major [n][dim] in original particle order,
 * fluid rows first, wall rows after them; r_ij = r_i - r_j (minimum image on
 * periodic axes); every neighbour sum runs over j in ascending index order.
 */
#ifndef SISPH_ORACLE_H
#define SISPH_ORACLE_H

#include <stdint.h>

enum { ORC_QUINTIC = 0, ORC_WENDLAND_C2 = 1 };
enum { ORC_ASYMM = 0, ORC_SYMM = 1 };
enum { ORC_GTVF_OFF = 0, ORC_GTVF_INTERNAL = 1, ORC_GTVF_EXTERNAL = 2 };
enum { ORC_PREF_FIXED = 0, ORC_PREF_TWICE_MAX = 1 };
enum { ORC_CONV_SUM = 0, ORC_CONV_MEAN = 1 };
enum { ORC_USTAR_SLIP = 0, ORC_USTAR_NOSLIP = 1 };
enum { ORC_DT_FIXED = 0, ORC_DT_ADAPTIVE = 1 };
enum { ORC_JACOBI = 0, ORC_BICGSTAB = 1 };
enum { ORC_NULL_NONE = 0, ORC_NULL_PROJECT = 1 };

typedef struct {
    int64_t dim, kernel, pgrad, gtvf, free_surface, p_ref_mode;
    int64_t min_iter, max_iter, gtvf_K, forced_iters, conv_norm, ustar_wall;
    int64_t dt_mode;  /* ORC_DT_FIXED: every step takes dt; ORC_DT_ADAPTIVE:
                         dt_next is chosen from this step's maxima */
    int64_t solver;   /* ORC_JACOBI (the paper's scheme) or ORC_BICGSTAB */
    int64_t null_space; /* ORC_NULL_PROJECT: on a fully periodic case (no
                           walls, no free surface) remove from the RHS its
                           component along the operator's left null vector
                           before the solve; ORC_NULL_NONE: as printed */
    int64_t nf, nw;
    double h, rho0, nu, alpha, c_ref, dt, eta, fs_ratio, omega, tol;
    double dt_max;    /* adaptive mode: upper bound of dt_next             */
    double g[3], lo[3], hi[3];
    int64_t periodic[3];
} orc_params;

/* Optional per-step outputs (any pointer may be NULL). */
typedef struct {
    double *rho;      /* [nf]       summation density at r^n               */
    double *xs;       /* [nf][dim]  r* (wrapped into the box)              */
    double *us;       /* [nf][dim]  u*                                     */
    double *uw;       /* [nw][dim]  wall velocity, no-slip form, at r^n    */
    double *usw;      /* [nw][dim]  wall u* at r* (the case's ghost form)  */
    double *rhs;      /* [nf]       PPE right-hand side                    */
    double *diag;     /* [nf]       D_ii                                   */
    double *unew;     /* [nf][dim]  u^{n+1}                                */
    double *fgtvf0;   /* [nf][dim]  GTVF acceleration at the first sub-step */
    int64_t *fs;      /* [nf]       free-surface flag                      */
    int64_t iters;    /* Jacobi sweeps done                                */
    int64_t converged;
    double ratio, lambda, p_ref_used;
    double beta;      /* the constant removed per unit D_ii from the RHS
                         (ORC_NULL_PROJECT), else 0                        */
    double umax;      /* max |u^n| over fluid particles                    */
    double fmax;      /* max |f^n|, f = predictor forces + pressure force  */
    double dt_next;   /* the next step's dt (dt itself in fixed mode)      */
} orc_step_out;

/* Kernel value and radial derivative dW/dr for smoothing length h. */
double orc_W(int64_t kernel, int64_t dim, double r, double h);
double orc_dWdr(int64_t kernel, int64_t dim, double r, double h);
double orc_support(int64_t kernel);

/* Threads of the per-row loops (1 in the serial build), and a setter
 * (ignored by the serial build). */
int64_t orc_threads(void);
void orc_set_threads(int64_t n);

/* Neighbour sets {j in [s0,s1) : |r_ij|^2 < R^2} for dest i in [d0,d1).
 * Brute force O(N^2) and cell-list variants; both return CSR with ids in
 * ascending order.  Return value = number of entries written, or -1 if cap
 * is too small (offsets are then still complete). */
int64_t orc_neighbors_brute(const orc_params *P, const double *x,
                            int64_t d0, int64_t d1, int64_t s0, int64_t s1,
                            int64_t *offsets, int32_t *ids, int64_t cap);
int64_t orc_neighbors_cells(const orc_params *P, const double *x,
                            int64_t d0, int64_t d1, int64_t s0, int64_t s1,
                            int64_t *offsets, int32_t *ids, int64_t cap);

/* Wall unit normals from positions only (section 3.4.1). */
void orc_wall_normals(const orc_params *P, const double *x, const double *m,
                      double *nrm);

/* Single operators at given positions, for the pins. Fluid dest only. */
void orc_density(const orc_params *P, const double *x, const double *m,
                 double *rho);
void orc_predictor_forces(const orc_params *P, const double *x,
                          const double *u_all, const double *ut,
                          const double *m, const double *rho_all, double *f);
void orc_ppe_operator(const orc_params *P, const double *x, const double *m,
                      const double *rho_all, const double *p_all,
                      double *lap, double *diag);
void orc_rhs(const orc_params *P, const double *x, const double *m,
             const double *rho_all, const double *us_all, double *rhs);
void orc_pressure_force(const orc_params *P, const double *x, const double *m,
                        const double *rho_all, const double *p_all, double *f);
void orc_gtvf_force(const orc_params *P, const double *x, const double *m,
                    const double *rho_all, const double *p0, double hgtvf,
                    double *f);
void orc_wall_pressure(const orc_params *P, const double *x,
                       const double *rho_all, double *p_all);
void orc_wall_velocity(const orc_params *P, const double *x,
                       const double *u_fluid, const double *wall_u,
                       const double *nrm, int64_t slip, double *uw);

/* One full SISPH step (the whole of Algorithm 1's loop body), in place.
 * x [nf+nw][dim], u [nf][dim], ut [nf][dim], p [nf+nw], m [nf+nw],
 * nrm [nw][dim], wall_u [nw][dim] (may be NULL: static walls).
 * p_ref is read and, in TWICE_MAX mode when *p_ref_set == 0, written after
 * the solve.  Returns 0. */
int64_t orc_step(const orc_params *P, double *x, double *u, double *ut,
                 double *p, const double *m, const double *nrm,
                 const double *wall_u, double *p_ref, int64_t *p_ref_set,
                 orc_step_out *out);

#endif
