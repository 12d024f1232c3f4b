/* SISPH oracle: plain serial FP64 reference of one SISPH time step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product library.  It shares no
 * source with the HIP path.  Every neighbour sum runs over the neighbour set
 * in ascending particle index; all arithmetic is IEEE double, compiled
 * without floating-point contraction (-ffp-contract=off) so that the
 * neighbour predicate |r_ij|^2 < R^2 and the position updates are exactly the
 * operations written here.
 *
 * Section / equation references are to Muta, Ramachandran & Negi,
 * arXiv:1908.01762.  Where the paper is silent or garbled the reading taken
 * is stated beside the code (readings R1..R19 are listed with the design
 * notes).
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include "sisph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ kernels
 * Quintic spline (Morris 1996, the "quintic spline" the paper uses for the
 * Taylor-Green and dam-break runs):
 *   W = s [ (3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5 ],  each term only where its
 *   bracket is positive; s = 7/(478 pi h^2) in 2D, 1/(120 pi h^3) in 3D.
 * Wendland C2: W = s (1 - q/2)^4 (2q + 1) for q < 2; s = 7/(4 pi h^2) in 2D,
 *   21/(16 pi h^3) in 3D.  q = r/h.                                          */
/* Threads the per-row loops use: the OpenMP build parallelises every loop
 * whose rows are independent (each row's neighbour sum stays serial, in
 * ascending neighbour order) and keeps every sum over rows serial, so its
 * results are bitwise those of the serial build. */
int64_t orc_threads(void) {
#ifdef _OPENMP
    return (int64_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int64_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}

double orc_support(int64_t kernel) { return kernel == ORC_QUINTIC ? 3.0 : 2.0; }

static double sigma(int64_t kernel, int64_t dim, double h) {
    if (kernel == ORC_QUINTIC)
        return dim == 2 ? 7.0 / (478.0 * PI * h * h) : 1.0 / (120.0 * PI * h * h * h);
    return dim == 2 ? 7.0 / (4.0 * PI * h * h) : 21.0 / (16.0 * PI * h * h * h);
}

static double pos5(double v) { return v > 0.0 ? v * v * v * v * v : 0.0; }
static double pos4(double v) { return v > 0.0 ? v * v * v * v : 0.0; }

double orc_W(int64_t kernel, int64_t dim, double r, double h) {
    double q = r / h, s = sigma(kernel, dim, h);
    if (kernel == ORC_QUINTIC)
        return s * (pos5(3.0 - q) - 6.0 * pos5(2.0 - q) + 15.0 * pos5(1.0 - q));
    if (q >= 2.0) return 0.0;
    double a = 1.0 - 0.5 * q;
    return s * a * a * a * a * (2.0 * q + 1.0);
}

double orc_dWdr(int64_t kernel, int64_t dim, double r, double h) {
    double q = r / h, s = sigma(kernel, dim, h);
    if (kernel == ORC_QUINTIC)
        return s / h * (-5.0 * pos4(3.0 - q) + 30.0 * pos4(2.0 - q) - 75.0 * pos4(1.0 - q));
    if (q >= 2.0) return 0.0;
    double a = 1.0 - 0.5 * q;
    /* d/dq [(1-q/2)^4 (2q+1)] = -5 q (1-q/2)^3 */
    return s / h * (-5.0 * q * a * a * a);
}

/* --------------------------------------------------------------- geometry */
/* r_ij = r_i - r_j, minimum image on periodic axes. */
static void pair_vec(const orc_params *P, const double *xi, const double *xj, double *d) {
    for (int k = 0; k < P->dim; ++k) {
        double v = xi[k] - xj[k];
        if (P->periodic[k]) {
            double L = P->hi[k] - P->lo[k];
            double Lh = 0.5 * L;
            if (v > Lh) v -= L;
            else if (v < -Lh) v += L;
        }
        d[k] = v;
    }
    for (int k = (int)P->dim; k < 3; ++k) d[k] = 0.0;
}

static double norm2(int64_t dim, const double *d) {
    double s = d[0] * d[0] + d[1] * d[1];
    if (dim == 3) s = s + d[2] * d[2];
    return s;
}

static double dot(int64_t dim, const double *a, const double *b) {
    double s = a[0] * b[0] + a[1] * b[1];
    if (dim == 3) s = s + a[2] * b[2];
    return s;
}

static double support_radius(const orc_params *P) { return orc_support(P->kernel) * P->h; }

/* Periodic wrap into [lo, hi). */
static double wrap1(double x, double lo, double hi) {
    double L = hi - lo;
    if (x >= hi) x -= L;
    else if (x < lo) {
        x += L;
        if (x >= hi) x = lo;
    }
    return x;
}

/* ---------------------------------------------------------- neighbour sets */
typedef struct {
    int64_t *off; /* [nd+1] */
    int32_t *ids;
} csr_t;

static void csr_free(csr_t *c) {
    free(c->off);
    free(c->ids);
    c->off = NULL;
    c->ids = NULL;
}

int64_t orc_neighbors_brute(const orc_params *P, const double *x,
                            int64_t d0, int64_t d1, int64_t s0, int64_t s1,
                            int64_t *offsets, int32_t *ids, int64_t cap) {
    double R = support_radius(P), R2 = R * R, d[3];
    int64_t dim = P->dim, cnt = 0;
    int overflow = 0;
    offsets[0] = 0;
    for (int64_t i = d0; i < d1; ++i) {
        for (int64_t j = s0; j < s1; ++j) {
            pair_vec(P, x + i * dim, x + j * dim, d);
            if (norm2(dim, d) < R2) {
                if (cnt < cap) ids[cnt] = (int32_t)j;
                else overflow = 1;
                ++cnt;
            }
        }
        offsets[i - d0 + 1] = cnt;
    }
    return overflow ? -1 : cnt;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int64_t cell_coord(double xv, double lo, double edge, int64_t n) {
    int64_t c = (int64_t)floor((xv - lo) / edge);
    if (c < 0) c = 0;
    if (c > n - 1) c = n - 1;
    return c;
}

/* Uniform grid with cell edge >= R; a particle outside a non-periodic box is
 * put in the nearest edge cell.  Candidates come from the 3^dim cells around
 * the particle's cell (each visited once), are tested with the exact
 * predicate and sorted ascending. */
static csr_t build_cells(const orc_params *P, const double *x,
                         int64_t d0, int64_t d1, int64_t s0, int64_t s1) {
    int64_t dim = P->dim, nc[3] = {1, 1, 1};
    double R = support_radius(P), R2 = R * R, edge[3] = {1, 1, 1};
    for (int k = 0; k < dim; ++k) {
        double L = P->hi[k] - P->lo[k];
        /* a small margin keeps the edge above R after rounding, so that
         * two particles closer than R are never two cells apart */
        nc[k] = (int64_t)floor(L / (R * 1.000001));
        if (nc[k] < 1) nc[k] = 1;
        edge[k] = L / (double)nc[k];
        if (edge[k] < R * 1.000001) edge[k] = R * 1.000001;
    }
    int64_t ncell = nc[0] * nc[1] * nc[2], ns = s1 - s0;
    int64_t *start = calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cellof = malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    int32_t *items = malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
    for (int64_t j = s0; j < s1; ++j) {
        int64_t c[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) c[k] = cell_coord(x[j * dim + k], P->lo[k], edge[k], nc[k]);
        cellof[j - s0] = (c[2] * nc[1] + c[1]) * nc[0] + c[0];
        start[cellof[j - s0] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    memcpy(fill, start, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t j = s0; j < s1; ++j) items[fill[cellof[j - s0]]++] = (int32_t)j;
    free(fill);

    int64_t nd = d1 - d0;
    csr_t out;
    out.off = malloc(sizeof(int64_t) * (size_t)(nd + 1));
    out.ids = NULL;
    out.off[0] = 0;
    /* two passes over the destination rows, each row independent of the
     * others: count the accepted candidates, then, after a prefix sum,
     * write them and sort each row ascending */
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < nd; ++i) out.off[i + 1] += out.off[i];
            out.ids = malloc(sizeof(int32_t) * (size_t)(out.off[nd] > 0 ? out.off[nd] : 1));
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = d0; i < d1; ++i) {
            double d[3];
            int64_t ci[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) ci[k] = cell_coord(x[i * dim + k], P->lo[k], edge[k], nc[k]);
            /* candidate cell coordinates per axis, deduplicated */
            int64_t cand[3][3], ncand[3] = {1, 1, 1};
            for (int k = 0; k < 3; ++k) cand[k][0] = 0;
            for (int k = 0; k < dim; ++k) {
                ncand[k] = 0;
                for (int o = -1; o <= 1; ++o) {
                    int64_t c = ci[k] + o;
                    if (P->periodic[k]) c = (c % nc[k] + nc[k]) % nc[k];
                    else if (c < 0 || c >= nc[k]) continue;
                    int dup = 0;
                    for (int t = 0; t < ncand[k]; ++t) dup |= (cand[k][t] == c);
                    if (!dup) cand[k][ncand[k]++] = c;
                }
            }
            int64_t cnt = 0, row0 = pass == 1 ? out.off[i - d0] : 0;
            for (int a = 0; a < ncand[2]; ++a)
                for (int b = 0; b < ncand[1]; ++b)
                    for (int e = 0; e < ncand[0]; ++e) {
                        int64_t cell = (cand[2][a] * nc[1] + cand[1][b]) * nc[0] + cand[0][e];
                        for (int64_t t = start[cell]; t < start[cell + 1]; ++t) {
                            int32_t j = items[t];
                            pair_vec(P, x + i * dim, x + (int64_t)j * dim, d);
                            if (norm2(dim, d) < R2) {
                                if (pass == 1) out.ids[row0 + cnt] = j;
                                ++cnt;
                            }
                        }
                    }
            if (pass == 0) out.off[i - d0 + 1] = cnt;
            else qsort(out.ids + row0, (size_t)cnt, sizeof(int32_t), cmp_i32);
        }
    }
    free(start);
    free(cellof);
    free(items);
    return out;
}

int64_t orc_neighbors_cells(const orc_params *P, const double *x,
                            int64_t d0, int64_t d1, int64_t s0, int64_t s1,
                            int64_t *offsets, int32_t *ids, int64_t cap) {
    csr_t c = build_cells(P, x, d0, d1, s0, s1);
    int64_t nd = d1 - d0, tot = c.off[nd];
    memcpy(offsets, c.off, sizeof(int64_t) * (size_t)(nd + 1));
    memcpy(ids, c.ids, sizeof(int32_t) * (size_t)(tot < cap ? tot : cap));
    csr_free(&c);
    return tot <= cap ? tot : -1;
}

/* Kernel gradient grad_i W(r_ij, h) = W'(r) r_ij / r (zero at r = 0). */
static void grad_w(const orc_params *P, const double *rij, double r, double h, double *g) {
    double dw = r > 0.0 ? orc_dWdr(P->kernel, P->dim, r, h) / r : 0.0;
    for (int k = 0; k < 3; ++k) g[k] = dw * rij[k];
}

/* ------------------------------------------------------------- operators */

/* Summation density, eq. summation_density (section 2.1). */
static void density_c(const orc_params *P, const csr_t *N, const double *x,
                      const double *m, double *rho) {
    int64_t dim = P->dim;
    double d[3];
#pragma omp parallel for schedule(static) private(d)
    for (int64_t i = 0; i < P->nf; ++i) {
        double s = 0.0;
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e) {
            int64_t j = N->ids[e];
            pair_vec(P, x + i * dim, x + j * dim, d);
            s += m[j] * orc_W(P->kernel, dim, sqrt(norm2(dim, d)), P->h);
        }
        rho[i] = s;
    }
}

/* Wall velocity (section 3.4): Shepard average of the fluid velocity with a
 * kernel of half the smoothing length (eq. vf); no-slip ghost velocity
 * 2 u_wall - u_avg (eq. vg-adami) or, in the slip form used for u*, the
 * average itself (reading R12); then any component into the solid is removed
 * (eq. vg-no-normal).  Nw = wall -> fluid neighbour sets. */
static void wall_velocity_c(const orc_params *P, const csr_t *Nw, const double *x,
                            const double *u_fluid, const double *wall_u,
                            const double *nrm, int64_t slip, double *uw) {
    int64_t dim = P->dim;
    double d[3];
#pragma omp parallel for schedule(static) private(d)
    for (int64_t w = 0; w < P->nw; ++w) {
        int64_t iw = P->nf + w;
        double num[3] = {0, 0, 0}, den = 0.0;
        for (int64_t e = Nw->off[w]; e < Nw->off[w + 1]; ++e) {
            int64_t f = Nw->ids[e];
            pair_vec(P, x + iw * dim, x + f * dim, d);
            double W = orc_W(P->kernel, dim, sqrt(norm2(dim, d)), 0.5 * P->h);
            for (int k = 0; k < dim; ++k) num[k] += u_fluid[f * dim + k] * W;
            den += W;
        }
        double v[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            double avg = den > 0.0 ? num[k] / den : 0.0;
            double uwall = wall_u ? wall_u[w * dim + k] : 0.0;
            v[k] = slip ? avg : 2.0 * uwall - avg;
        }
        double vn = dot(dim, v, nrm + w * dim);
        if (vn < 0.0)
            for (int k = 0; k < dim; ++k) v[k] -= vn * nrm[w * dim + k];
        for (int k = 0; k < dim; ++k) uw[w * dim + k] = v[k];
    }
}

/* Predictor accelerations at r^n (eq. mom:sph without f_p):
 *   viscous   eq. mom:sph:visc
 *   art. visc eq. mom:sph:av / av:params, read as Monaghan's form
 *             Pi_ij = -alpha h c_ref mu_ij / rho_bar when u_ij.r_ij < 0,
 *             mu_ij = u_ij.r_ij / (r^2 + eta h^2), force -sum m_j Pi_ij gradW
 *             (reading R9)
 *   art. stress eq. mom:sph:gtvf:stress with the mass and kernel gradient the
 *             printed form drops: sum m_j (A_i/rho_i^2 + A_j/rho_j^2) . gradW,
 *             A = rho u (x) (u_tilde - u), A = 0 on walls (reading R8)
 *   body force g.
 * u_all: [nf+nw][dim] (fluid velocity, then wall ghost velocity). */
static void forces_c(const orc_params *P, const csr_t *N, const double *x,
                     const double *u_all, const double *ut, const double *m,
                     const double *rho_all, double *f) {
    int64_t dim = P->dim;
    double epsh = P->eta * P->h * P->h, d[3], g[3];
#pragma omp parallel for schedule(static) private(d, g)
    for (int64_t i = 0; i < P->nf; ++i) {
        double fv[3] = {0, 0, 0}, fa[3] = {0, 0, 0}, fs[3] = {0, 0, 0};
        double Ai[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Ai[a][b] = (a < dim && b < dim)
                               ? rho_all[i] * u_all[i * dim + a] * (ut[i * dim + b] - u_all[i * dim + b])
                               : 0.0;
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e) {
            int64_t j = N->ids[e];
            pair_vec(P, x + i * dim, x + j * dim, d);
            double r2 = norm2(dim, d), r = sqrt(r2);
            grad_w(P, d, r, P->h, g);
            double F = dot(dim, d, g);
            double uij[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) uij[k] = u_all[i * dim + k] - u_all[j * dim + k];
            /* viscous */
            double cv = m[j] * 4.0 * P->nu / (rho_all[i] + rho_all[j]) * F / (r2 + epsh);
            for (int k = 0; k < dim; ++k) fv[k] += cv * uij[k];
            /* artificial viscosity */
            double vr = dot(dim, uij, d);
            if (vr < 0.0 && P->alpha > 0.0) {
                double mu = vr / (r2 + epsh);
                double rhobar = 0.5 * (rho_all[i] + rho_all[j]);
                double Pi = -P->alpha * P->h * P->c_ref * mu / rhobar;
                for (int k = 0; k < dim; ++k) fa[k] -= m[j] * Pi * g[k];
            }
            /* artificial stress */
            double Aj[3][3] = {{0}};
            if (j < P->nf)
                for (int a = 0; a < dim; ++a)
                    for (int b = 0; b < dim; ++b)
                        Aj[a][b] = rho_all[j] * u_all[j * dim + a] * (ut[j * dim + b] - u_all[j * dim + b]);
            double ri2 = rho_all[i] * rho_all[i], rj2 = rho_all[j] * rho_all[j];
            for (int a = 0; a < dim; ++a) {
                double s = 0.0;
                for (int b = 0; b < dim; ++b) s += (Ai[a][b] / ri2 + Aj[a][b] / rj2) * g[b];
                fs[a] += m[j] * s;
            }
        }
        for (int k = 0; k < dim; ++k) f[i * dim + k] = fv[k] + fa[k] + fs[k] + P->g[k];
    }
}

/* PPE right-hand side and coefficients (eqs. sph-ppe, coeff, coeff1) at r*:
 *   RHS_i = sum -m_j/(rho_j dt) u*_ij . grad_i W_ij
 *   c_ij  = 4 m_j / (rho_i (rho_i + rho_j)) * (r_ij . grad_i W_ij) / (r^2 + eta h^2)
 *   D_ii  = sum_j c_ij,  and OD_ij = -c_ij.
 * The printed coefficient denominator "r^2 + eta^2" is read as r^2 + eta h^2,
 * as in eq. sph-ppe and the coefficient listing (reading R1). */
static void rhs_coef_c(const orc_params *P, const csr_t *N, const double *x,
                       const double *m, const double *rho_all, const double *us_all,
                       double *rhs, double *coef, double *diag) {
    int64_t dim = P->dim;
    double epsh = P->eta * P->h * P->h, d[3], g[3];
#pragma omp parallel for schedule(static) private(d, g)
    for (int64_t i = 0; i < P->nf; ++i) {
        double s = 0.0, D = 0.0;
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e) {
            int64_t j = N->ids[e];
            pair_vec(P, x + i * dim, x + j * dim, d);
            double r2 = norm2(dim, d), r = sqrt(r2);
            grad_w(P, d, r, P->h, g);
            double usij[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) usij[k] = us_all[i * dim + k] - us_all[j * dim + k];
            s += -m[j] / (rho_all[j] * P->dt) * dot(dim, usij, g);
            double c = 4.0 * m[j] / (rho_all[i] * (rho_all[i] + rho_all[j])) * dot(dim, d, g) / (r2 + epsh);
            if (coef) coef[e] = c;
            D += c;
        }
        rhs[i] = s;
        diag[i] = D;
    }
}

/* Fully periodic problems without walls or a free surface (the Taylor-Green
 * vortex): every row of eq. sph-ppe sums c_ij (p_j - p_i), so a constant
 * pressure solves the homogeneous system and the operator A = D - C is
 * singular.  Because m_i rho_i c_ij is symmetric in i and j, y_i = m_i rho_i
 * is a left null vector (y^T A = 0): the system has a solution only when
 * y . RHS = 0.  The discrete RHS does not satisfy this exactly (its pair
 * terms are not antisymmetric on a disordered set), and then each Jacobi
 * sweep of eq. p-sor shifts the iterate by the same constant w beta, with
 * beta = (y . RHS) / (y . D); the shift never settles, and the stopping test
 * of eq. convergence sees it as a change of the pressure.  Reading R24
 * removes that component once per solve, RHS_i <- RHS_i - beta D_ii; every
 * iterate then equals the unprojected one minus k w beta after k sweeps
 * (eq. p-sor maps p + c to its image + c), so only the constant, to which
 * the asymm pressure force is blind, changes.  Returns beta. */
static double project_rhs_c(const orc_params *P, const double *m, const double *rho_all,
                            double *rhs, const double *diag) {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < P->nf; ++i) {
        double y = m[i] * rho_all[i];
        num += y * rhs[i];
        den += y * diag[i];
    }
    double beta = den != 0.0 ? num / den : 0.0;
    for (int64_t i = 0; i < P->nf; ++i)
        if (diag[i] != 0.0) rhs[i] -= beta * diag[i];
    return beta;
}

/* Solid-wall pressure, eq. p-shepard: Shepard average of the fluid pressure
 * plus the hydrostatic term (g - a_w) . sum rho_f r_wf W_wf, static wall so
 * a_w = 0; zero when no fluid neighbour; clamped at 0 on free-surface
 * problems (section 3.4).  Writes p_all[nf..nf+nw). */
static void wall_pressure_c(const orc_params *P, const csr_t *Nw, const double *x,
                            const double *rho_all, double *p_all) {
    int64_t dim = P->dim;
    double d[3];
#pragma omp parallel for schedule(static) private(d)
    for (int64_t w = 0; w < P->nw; ++w) {
        int64_t iw = P->nf + w;
        double sp = 0.0, sr[3] = {0, 0, 0}, sw = 0.0;
        for (int64_t e = Nw->off[w]; e < Nw->off[w + 1]; ++e) {
            int64_t f = Nw->ids[e];
            pair_vec(P, x + iw * dim, x + f * dim, d); /* r_wf = r_w - r_f */
            double W = orc_W(P->kernel, dim, sqrt(norm2(dim, d)), P->h);
            sp += p_all[f] * W;
            for (int k = 0; k < dim; ++k) sr[k] += rho_all[f] * d[k] * W;
            sw += W;
        }
        double pw = 0.0;
        if (sw > 0.0) pw = (sp + dot(dim, P->g, sr)) / sw;
        if (P->free_surface && pw < 0.0) pw = 0.0;
        p_all[iw] = pw;
    }
}

/* The linear part of eq. p-shepard (no hydrostatic term, no clamp):
 * z_w = sum_f z_f W_wf / sum_f W_wf, 0 without fluid neighbours.  Writes
 * z[nf..nf+nw).  With z = 0 for every fluid particle and hydro set, the
 * hydrostatic part alone instead. */
static void wall_extrap_c(const orc_params *P, const csr_t *Nw, const double *x,
                          const double *rho_all, double *z, int hydro) {
    int64_t dim = P->dim;
    double d[3];
#pragma omp parallel for schedule(static) private(d)
    for (int64_t w = 0; w < P->nw; ++w) {
        int64_t iw = P->nf + w;
        double sp = 0.0, sr[3] = {0, 0, 0}, sw = 0.0;
        for (int64_t e = Nw->off[w]; e < Nw->off[w + 1]; ++e) {
            int64_t f = Nw->ids[e];
            pair_vec(P, x + iw * dim, x + f * dim, d);
            double W = orc_W(P->kernel, dim, sqrt(norm2(dim, d)), P->h);
            sp += z[f] * W;
            for (int k = 0; k < dim; ++k) sr[k] += rho_all[f] * d[k] * W;
            sw += W;
        }
        z[iw] = sw > 0.0 ? (hydro ? dot(dim, P->g, sr) : sp) / sw : 0.0;
    }
}

/* BiCGStab (van der Vorst 1992) on the PPE scaled by its diagonal: for a
 * row i with D_ii != 0 that is not on the free surface,
 *   (M z)_i = z_i - sum_j c_ij z_j / D_ii,   f_i = (RHS_i + sum_w c_iw h_w) / D_ii
 * where a wall neighbour's value is the linear part of eq. p-shepard applied
 * to z and h_w its hydrostatic part; every other row is z_i = 0.  Starts from
 * p^n.  After iteration k the stopping test is eq. convergence with the
 * Jacobi update replaced by omega times the scaled residual (the update a
 * Jacobi sweep from x_k would make): omega sum|r_k| / max(Lambda, sum|x_k|)
 * < tol, or k >= max_iter (forced_iters > 0: exactly that many).  A zero
 * denominator in a step coefficient stops the iteration after that step.
 * Only free-surface problems are solved this way: without free-surface
 * (p = 0) rows every row of M annihilates constants, the system fixes p only
 * up to one and BiCGStab drifts along it (the caller refuses those).
 * On return p[0..nf) holds the solution; *iters and *ratio are set. */
static void bicgstab_c(const orc_params *P, const csr_t *N, const csr_t *Nw, const double *xs,
                       const double *rho_all, const double *coef, const double *diag,
                       const double *rhs, const int64_t *fs, double lambda, double *p,
                       int64_t *iters, double *ratio_out) {
    int64_t nf = P->nf, n = nf + P->nw;
    size_t n1 = (size_t)(n > 0 ? n : 1);
    double *h = calloc(n1, sizeof(double)), *f = calloc(n1, sizeof(double));
    double *x = calloc(n1, sizeof(double)), *r = calloc(n1, sizeof(double));
    double *rh = calloc(n1, sizeof(double)), *pv = calloc(n1, sizeof(double));
    double *v = calloc(n1, sizeof(double)), *sv = calloc(n1, sizeof(double));
    double *t = calloc(n1, sizeof(double)), *mx = calloc(n1, sizeof(double));
    char *act = calloc(n1, 1);
    for (int64_t i = 0; i < nf; ++i) act[i] = diag[i] != 0.0 && !fs[i];
    if (P->nw) wall_extrap_c(P, Nw, xs, rho_all, h, 1);
    /* (M z) for the fluid rows; the wall slots of z must hold its extrapolation */
#define APPLY_M(z, out)                                                        \
    _Pragma("omp parallel for schedule(static)")                               \
    for (int64_t i = 0; i < nf; ++i) {                                         \
        if (!act[i]) { (out)[i] = (z)[i]; continue; }                          \
        double acc = 0.0;                                                      \
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e)                    \
            acc += coef[e] * (z)[N->ids[e]];                                   \
        (out)[i] = (z)[i] - acc / diag[i];                                     \
    }
    for (int64_t i = 0; i < nf; ++i) {
        if (!act[i]) continue;
        double acc = 0.0;
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e)
            if (N->ids[e] >= nf) acc += coef[e] * h[N->ids[e]];
        f[i] = (rhs[i] + acc) / diag[i];
        x[i] = p[i];
    }
    if (P->nw) wall_extrap_c(P, Nw, xs, rho_all, x, 0);
    APPLY_M(x, mx);
    for (int64_t i = 0; i < nf; ++i) {
        r[i] = act[i] ? f[i] - mx[i] : 0.0;
        rh[i] = r[i];
    }
    double rho_old = 1.0, alpha = 1.0, om = 1.0, ratio = 0.0;
    double lam_s = P->conv_norm == ORC_CONV_MEAN ? (double)nf * lambda : lambda;
    int64_t k = 0;
    for (;;) {
        double rho = 0.0;
        for (int64_t i = 0; i < nf; ++i) rho += rh[i] * r[i];
        double beta = (rho / rho_old) * (alpha / om);
        for (int64_t i = 0; i < nf; ++i) pv[i] = r[i] + beta * (pv[i] - om * v[i]);
        if (P->nw) wall_extrap_c(P, Nw, xs, rho_all, pv, 0);
        APPLY_M(pv, v);
        double rv = 0.0;
        for (int64_t i = 0; i < nf; ++i) rv += rh[i] * v[i];
        int brk = rv == 0.0;
        alpha = brk ? 0.0 : rho / rv;
        for (int64_t i = 0; i < nf; ++i) sv[i] = r[i] - alpha * v[i];
        if (P->nw) wall_extrap_c(P, Nw, xs, rho_all, sv, 0);
        APPLY_M(sv, t);
        double ts = 0.0, tt = 0.0;
        for (int64_t i = 0; i < nf; ++i) {
            ts += t[i] * sv[i];
            tt += t[i] * t[i];
        }
        brk = brk || tt == 0.0;
        om = tt == 0.0 ? 0.0 : ts / tt;
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < nf; ++i) {
            x[i] = x[i] + alpha * pv[i] + om * sv[i];
            r[i] = sv[i] - om * t[i];
            num += fabs(r[i]);
            den += fabs(x[i]);
        }
        num *= P->omega;
        double scale = lam_s > den ? lam_s : den;
        ratio = scale > 0.0 ? num / scale : (num > 0.0 ? INFINITY : 0.0);
        ++k;
        rho_old = rho;
        if (P->forced_iters > 0) {
            if (k >= P->forced_iters) break;
        } else if (ratio < P->tol || k >= P->max_iter || brk || !isfinite(num) || !isfinite(den)) {
            break;
        }
    }
#undef APPLY_M
    for (int64_t i = 0; i < nf; ++i) p[i] = x[i];
    *iters = k;
    *ratio_out = ratio;
    free(h); free(f); free(x); free(r); free(rh); free(pv); free(v); free(sv); free(t); free(mx); free(act);
}

/* Pressure acceleration, eq. mom:sph:press:pij (asymm) or
 * eq. mom:sph:press:symm (symm). */
static void pressure_force_c(const orc_params *P, const csr_t *N, const double *x,
                             const double *m, const double *rho_all, const double *p_all,
                             double *f) {
    int64_t dim = P->dim;
    double d[3], g[3];
#pragma omp parallel for schedule(static) private(d, g)
    for (int64_t i = 0; i < P->nf; ++i) {
        double a[3] = {0, 0, 0};
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e) {
            int64_t j = N->ids[e];
            pair_vec(P, x + i * dim, x + j * dim, d);
            double r = sqrt(norm2(dim, d));
            grad_w(P, d, r, P->h, g);
            double c;
            if (P->pgrad == ORC_SYMM)
                c = -m[j] * (p_all[i] / (rho_all[i] * rho_all[i]) + p_all[j] / (rho_all[j] * rho_all[j]));
            else
                c = -m[j] / (rho_all[i] * rho_all[j]) * (p_all[j] - p_all[i]);
            for (int k = 0; k < dim; ++k) a[k] += c * g[k];
        }
        for (int k = 0; k < dim; ++k) f[i * dim + k] = a[k];
    }
}

/* GTVF background-pressure acceleration, eq. mom:sph:gtvf:
 * f_i = -p0_i sum_j m_j / rho_j^2 grad_i W(r_ij, h_tilde). */
static void gtvf_force_c(const orc_params *P, const csr_t *N, const double *x,
                         const double *m, const double *rho_all, const double *p0,
                         double ht, double *f) {
    int64_t dim = P->dim;
    double d[3], g[3];
#pragma omp parallel for schedule(static) private(d, g)
    for (int64_t i = 0; i < P->nf; ++i) {
        double a[3] = {0, 0, 0};
        for (int64_t e = N->off[i]; e < N->off[i + 1]; ++e) {
            int64_t j = N->ids[e];
            pair_vec(P, x + i * dim, x + j * dim, d);
            double r = sqrt(norm2(dim, d));
            grad_w(P, d, r, ht, g);
            double c = m[j] / (rho_all[j] * rho_all[j]);
            for (int k = 0; k < dim; ++k) a[k] += c * g[k];
        }
        for (int k = 0; k < dim; ++k) f[i * dim + k] = -p0[i] * a[k];
    }
}

/* ----------------------------------------------------- public operators */
static csr_t fluid_nbrs(const orc_params *P, const double *x) {
    return build_cells(P, x, 0, P->nf, 0, P->nf + P->nw);
}
static csr_t wall_nbrs(const orc_params *P, const double *x) {
    return build_cells(P, x, P->nf, P->nf + P->nw, 0, P->nf);
}

void orc_density(const orc_params *P, const double *x, const double *m, double *rho) {
    csr_t N = fluid_nbrs(P, x);
    density_c(P, &N, x, m, rho);
    csr_free(&N);
}

void orc_predictor_forces(const orc_params *P, const double *x, const double *u_all,
                          const double *ut, const double *m, const double *rho_all,
                          double *f) {
    csr_t N = fluid_nbrs(P, x);
    forces_c(P, &N, x, u_all, ut, m, rho_all, f);
    csr_free(&N);
}

void orc_ppe_operator(const orc_params *P, const double *x, const double *m,
                      const double *rho_all, const double *p_all, double *lap,
                      double *diag) {
    csr_t N = fluid_nbrs(P, x);
    int64_t nf = P->nf, n = nf + P->nw, dim = P->dim;
    double *coef = malloc(sizeof(double) * (size_t)(N.off[nf] > 0 ? N.off[nf] : 1));
    double *rhs = malloc(sizeof(double) * (size_t)(nf > 0 ? nf : 1));
    double *zu = calloc((size_t)(n * dim > 0 ? n * dim : 1), sizeof(double));
    rhs_coef_c(P, &N, x, m, rho_all, zu, rhs, coef, diag);
    /* sum_j c_ij (p_i - p_j): the discrete operator of eq. sph-ppe */
    for (int64_t i = 0; i < nf; ++i) {
        double s = 0.0;
        for (int64_t e = N.off[i]; e < N.off[i + 1]; ++e) s += coef[e] * (p_all[i] - p_all[N.ids[e]]);
        lap[i] = s;
    }
    free(coef);
    free(rhs);
    free(zu);
    csr_free(&N);
}

void orc_rhs(const orc_params *P, const double *x, const double *m, const double *rho_all,
             const double *us_all, double *rhs) {
    csr_t N = fluid_nbrs(P, x);
    double *diag = malloc(sizeof(double) * (size_t)(P->nf > 0 ? P->nf : 1));
    rhs_coef_c(P, &N, x, m, rho_all, us_all, rhs, NULL, diag);
    free(diag);
    csr_free(&N);
}

void orc_pressure_force(const orc_params *P, const double *x, const double *m,
                        const double *rho_all, const double *p_all, double *f) {
    csr_t N = fluid_nbrs(P, x);
    pressure_force_c(P, &N, x, m, rho_all, p_all, f);
    csr_free(&N);
}

void orc_gtvf_force(const orc_params *P, const double *x, const double *m,
                    const double *rho_all, const double *p0, double hgtvf, double *f) {
    csr_t N = fluid_nbrs(P, x);
    gtvf_force_c(P, &N, x, m, rho_all, p0, hgtvf, f);
    csr_free(&N);
}

void orc_wall_pressure(const orc_params *P, const double *x, const double *rho_all,
                       double *p_all) {
    csr_t Nw = wall_nbrs(P, x);
    wall_pressure_c(P, &Nw, x, rho_all, p_all);
    csr_free(&Nw);
}

void orc_wall_velocity(const orc_params *P, const double *x, const double *u_fluid,
                       const double *wall_u, const double *nrm, int64_t slip, double *uw) {
    csr_t Nw = wall_nbrs(P, x);
    wall_velocity_c(P, &Nw, x, u_fluid, wall_u, nrm, slip, uw);
    csr_free(&Nw);
}

/* Wall normals from positions only (section 3.4.1, eqs. normal-approx and
 * normal), summed over wall neighbours only (reading R7), wall density rho0:
 *   n*_w = -sum_j (m_j/rho0) grad_w W_wj, zeroed when |n*| < 1/(4h), else
 *   made unit; n_w = sum_j (m_j/rho0) n*_j W_wj, made unit. */
void orc_wall_normals(const orc_params *P, const double *x, const double *m, double *nrm) {
    int64_t nf = P->nf, nw = P->nw, dim = P->dim;
    if (nw == 0) return;
    csr_t N = build_cells(P, x, nf, nf + nw, nf, nf + nw);
    double *ns = calloc((size_t)(nw * dim), sizeof(double));
    double d[3], g[3];
#pragma omp parallel for schedule(static) private(d, g)
    for (int64_t w = 0; w < nw; ++w) {
        int64_t iw = nf + w;
        double a[3] = {0, 0, 0};
        for (int64_t e = N.off[w]; e < N.off[w + 1]; ++e) {
            int64_t j = N.ids[e];
            pair_vec(P, x + iw * dim, x + j * dim, d);
            grad_w(P, d, sqrt(norm2(dim, d)), P->h, g);
            for (int k = 0; k < dim; ++k) a[k] -= m[j] / P->rho0 * g[k];
        }
        double mag = sqrt(dot(dim, a, a));
        for (int k = 0; k < dim; ++k) ns[w * dim + k] = mag < 1.0 / (4.0 * P->h) ? 0.0 : a[k] / mag;
    }
#pragma omp parallel for schedule(static) private(d)
    for (int64_t w = 0; w < nw; ++w) {
        int64_t iw = nf + w;
        double a[3] = {0, 0, 0};
        for (int64_t e = N.off[w]; e < N.off[w + 1]; ++e) {
            int64_t j = N.ids[e];
            pair_vec(P, x + iw * dim, x + j * dim, d);
            double W = orc_W(P->kernel, dim, sqrt(norm2(dim, d)), P->h);
            for (int k = 0; k < dim; ++k) a[k] += m[j] / P->rho0 * ns[(j - nf) * dim + k] * W;
        }
        /* a smoothed normal that is only the rounding residue of opposite
         * layers cancelling (length below 1e-9, against ~1 for a real
         * surface) has no direction: it is set to zero (reading R7) */
        double mag = sqrt(dot(dim, a, a));
        for (int k = 0; k < dim; ++k) nrm[w * dim + k] = mag > 1e-9 ? a[k] / mag : 0.0;
    }
    free(ns);
    csr_free(&N);
}

/* -------------------------------------------------------------- one step
 * Algorithm 1 (section 3.1) with the two-stage split of the implementation
 * notes (section 3.3): density and predictor forces at r^n; PPE, pressure
 * force and GTVF at r* (reading R4). */
int64_t orc_step(const orc_params *P, double *x, double *u, double *ut, double *p,
                 const double *m, const double *nrm, const double *wall_u,
                 double *p_ref, int64_t *p_ref_set, orc_step_out *out) {
    int64_t nf = P->nf, nw = P->nw, n = nf + nw, dim = P->dim;
    double dt = P->dt;
    /* R24 holds only where constants are the null space: no walls (their
     * hydrostatic term) and no free-surface rows (p = 0 there) */
    if (P->null_space == ORC_NULL_PROJECT && (nw > 0 || P->free_surface)) return -1;
    size_t nd = (size_t)(n * dim > 0 ? n * dim : 1), n1 = (size_t)(n > 0 ? n : 1);
    double *rho_all = malloc(sizeof(double) * n1);
    double *u_all = calloc(nd, sizeof(double));
    double *f = calloc(nd, sizeof(double));
    double *xs = malloc(sizeof(double) * nd);
    double *us_all = calloc(nd, sizeof(double));
    double *rhs = calloc(n1, sizeof(double));
    double *diag = calloc(n1, sizeof(double));
    double *pk = malloc(sizeof(double) * n1);
    double *pn = malloc(sizeof(double) * n1);
    int64_t *fs = calloc(n1, sizeof(int64_t));
    double *unew = calloc(nd, sizeof(double));

    /* step 1-2: neighbours and summation density at r^n; free-surface flag
     * rho_i / rho0 < fs_ratio on free-surface problems (section 3) */
    csr_t N = fluid_nbrs(P, x), Nw = wall_nbrs(P, x);
    density_c(P, &N, x, m, rho_all);
    for (int64_t w = 0; w < nw; ++w) rho_all[nf + w] = P->rho0;
    for (int64_t i = 0; i < nf; ++i) fs[i] = P->free_surface && (rho_all[i] / P->rho0 < P->fs_ratio);

    /* step 3: wall ghost velocity, no-slip form, for the predictor forces */
    memcpy(u_all, u, sizeof(double) * (size_t)(nf * dim));
    if (nw) wall_velocity_c(P, &Nw, x, u, wall_u, nrm, 0, u_all + nf * dim);
    if (out && out->uw) memcpy(out->uw, u_all + nf * dim, sizeof(double) * (size_t)(nw * dim));

    /* step 4-5: predictor, eqs. int:rnp1 and int:vint; walls stay put */
    forces_c(P, &N, x, u_all, ut, m, rho_all, f);
    memcpy(xs, x, sizeof(double) * (size_t)(n * dim));
    for (int64_t i = 0; i < nf; ++i)
        for (int k = 0; k < dim; ++k) {
            double v = x[i * dim + k] + dt * ut[i * dim + k];
            if (P->periodic[k]) v = wrap1(v, P->lo[k], P->hi[k]);
            xs[i * dim + k] = v;
            us_all[i * dim + k] = u[i * dim + k] + dt * f[i * dim + k];
        }
    csr_free(&N);
    csr_free(&Nw);

    /* step 6: neighbours at r*; wall u* in the slip form (default, reading
     * R12) or the no-slip form (the alternative compared in section 4.3) */
    N = fluid_nbrs(P, xs);
    Nw = wall_nbrs(P, xs);
    if (nw) wall_velocity_c(P, &Nw, xs, us_all, wall_u, nrm, P->ustar_wall == ORC_USTAR_NOSLIP ? 0 : 1,
                            us_all + nf * dim);

    /* step 7: RHS, coefficients, D_ii, Lambda (eq. convergence; |RHS/D| over
     * non-free-surface fluid with D != 0, reading R2) */
    double *coef = malloc(sizeof(double) * (size_t)(N.off[nf] > 0 ? N.off[nf] : 1));
    rhs_coef_c(P, &N, xs, m, rho_all, us_all, rhs, coef, diag);
    double beta = 0.0;
    if (P->null_space == ORC_NULL_PROJECT) beta = project_rhs_c(P, m, rho_all, rhs, diag);
    double lambda = 0.0;
    for (int64_t i = 0; i < nf; ++i)
        if (diag[i] != 0.0 && !fs[i]) {
            double v = fabs(rhs[i] / diag[i]);
            if (v > lambda) lambda = v;
        }

    /* step 8: damped Jacobi ("SOR" with omega) from p^n, eq. p-sor; walls by
     * eq. p-shepard before every sweep; convergence by eq. convergence */
    memcpy(pk, p, sizeof(double) * (size_t)n);
    int64_t k = 0;
    double ratio = 0.0;
    if (P->solver == ORC_BICGSTAB && !P->free_surface) {
        /* refused: see bicgstab_c */
        k = -1;
        ratio = NAN;
    } else if (P->solver == ORC_BICGSTAB) bicgstab_c(P, &N, &Nw, xs, rho_all, coef, diag, rhs, fs, lambda, pk, &k, &ratio);
    else for (;;) {
        if (nw) wall_pressure_c(P, &Nw, xs, rho_all, pk);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nf; ++i) {
            double v = 0.0;
            if (diag[i] != 0.0 && !fs[i]) {
                double s = 0.0;
                for (int64_t e = N.off[i]; e < N.off[i + 1]; ++e) s += coef[e] * pk[N.ids[e]];
                v = P->omega * (rhs[i] + s) / diag[i] + (1.0 - P->omega) * pk[i];
            }
            pn[i] = v;
        }
        /* the two sums in row order, whatever the thread count */
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < nf; ++i) {
            num += fabs(pn[i] - pk[i]);
            den += fabs(pn[i]);
        }
        /* printed form: max(Lambda, sum|p|); the "mean" reading scales Lambda
         * by the fluid count so both terms measure a per-particle pressure */
        double lam_s = P->conv_norm == ORC_CONV_MEAN ? (double)nf * lambda : lambda;
        double scale = lam_s > den ? lam_s : den;
        ratio = scale > 0.0 ? num / scale : (num > 0.0 ? INFINITY : 0.0);
        memcpy(pk, pn, sizeof(double) * (size_t)nf);
        ++k;
        if (P->forced_iters > 0) {
            if (k >= P->forced_iters) break;
        } else if ((k >= P->min_iter && ratio < P->tol) || k >= P->max_iter) {
            break;
        }
    }
    if (nw) wall_pressure_c(P, &Nw, xs, rho_all, pk);

    /* p_ref for internal flows: twice the largest pressure after the first
     * solve, then held (section 2.1, reading R5) */
    if (P->p_ref_mode == ORC_PREF_TWICE_MAX && !*p_ref_set) {
        double mx = -INFINITY;
        for (int64_t i = 0; i < nf; ++i) mx = pk[i] > mx ? pk[i] : mx;
        *p_ref = 2.0 * mx;
        *p_ref_set = 1;
    }

    /* step 9: pressure acceleration and correction, eq. int:vnp1 */
    double *fp = calloc(nd, sizeof(double));
    pressure_force_c(P, &N, xs, m, rho_all, pk, fp);
    for (int64_t i = 0; i < nf; ++i)
        for (int kk = 0; kk < dim; ++kk)
            unew[i * dim + kk] = us_all[i * dim + kk] + dt * fp[i * dim + kk];

    /* the next step's dt (section 3.2, adaptive steps): the largest fluid
     * speed at the start of this step and the largest total acceleration
     * of this step (predictor forces with gravity, plus the pressure
     * force) */
    double umax2 = 0.0, fmax2 = 0.0;
    for (int64_t i = 0; i < nf; ++i) {
        double a = 0.0, b = 0.0;
        for (int kk = 0; kk < dim; ++kk) {
            double ui = u[i * dim + kk], fi = f[i * dim + kk] + fp[i * dim + kk];
            a += ui * ui;
            b += fi * fi;
        }
        if (a > umax2) umax2 = a;
        if (b > fmax2) fmax2 = b;
    }
    double umax = sqrt(umax2), fmax = sqrt(fmax2);
    double dt_next = dt;
    if (P->dt_mode == ORC_DT_ADAPTIVE) {
        dt_next = P->dt_max;
        if (umax > 0.0 && 0.25 * P->h / umax < dt_next) dt_next = 0.25 * P->h / umax;
        if (fmax > 0.0 && 0.25 * sqrt(P->h / fmax) < dt_next) dt_next = 0.25 * sqrt(P->h / fmax);
    }

    /* step 10: GTVF sub-steps on the frozen r* neighbour sets
     * (eqs. int:gtvf:pos, int:gtvf:vel:tmp); walls fixed; no wrap inside */
    double *xk = malloc(sizeof(double) * nd);
    double *vk = calloc(nd, sizeof(double));
    double *fk = calloc(nd, sizeof(double));
    double *p0 = calloc(n1, sizeof(double));
    memcpy(xk, xs, sizeof(double) * (size_t)(n * dim));
    if (P->gtvf != ORC_GTVF_OFF) {
        double ht = P->gtvf == ORC_GTVF_EXTERNAL ? 0.5 * P->h : P->h;
        for (int64_t i = 0; i < nf; ++i) {
            double a = 10.0 * fabs(pk[i]);
            p0[i] = P->gtvf == ORC_GTVF_EXTERNAL ? (a < *p_ref ? a : *p_ref) : *p_ref;
        }
        int64_t K = P->gtvf_K;
        double dtau = dt / (double)K;
        for (int64_t s = 0; s < K; ++s) {
            gtvf_force_c(P, &N, xk, m, rho_all, p0, ht, fk);
            if (s == 0 && out && out->fgtvf0) memcpy(out->fgtvf0, fk, sizeof(double) * (size_t)(nf * dim));
            for (int64_t i = 0; i < nf; ++i)
                for (int kk = 0; kk < dim; ++kk) {
                    int64_t q = i * dim + kk;
                    xk[q] = xk[q] + dtau * vk[q] + 0.5 * dtau * dtau * fk[q];
                    vk[q] = vk[q] + dtau * fk[q];
                }
        }
    }

    /* step 11: transport velocity and position update, eqs. int:vhatnp2 and
     * int:rnp2, then the periodic wrap; p^{n+1} = final iterate */
    for (int64_t i = 0; i < nf; ++i)
        for (int kk = 0; kk < dim; ++kk) {
            int64_t q = i * dim + kk;
            double utn = unew[q] + (xk[q] - xs[q]) / dt;
            double xn = x[q] + 0.5 * dt * (utn + ut[q]);
            if (P->periodic[kk]) xn = wrap1(xn, P->lo[kk], P->hi[kk]);
            x[q] = xn;
            ut[q] = utn;
            u[q] = unew[q];
        }
    memcpy(p, pk, sizeof(double) * (size_t)n);

    if (out) {
        if (out->rho) memcpy(out->rho, rho_all, sizeof(double) * (size_t)nf);
        if (out->xs) memcpy(out->xs, xs, sizeof(double) * (size_t)(nf * dim));
        if (out->us) memcpy(out->us, us_all, sizeof(double) * (size_t)(nf * dim));
        if (out->usw) memcpy(out->usw, us_all + nf * dim, sizeof(double) * (size_t)(nw * dim));
        if (out->rhs) memcpy(out->rhs, rhs, sizeof(double) * (size_t)nf);
        if (out->diag) memcpy(out->diag, diag, sizeof(double) * (size_t)nf);
        if (out->unew) memcpy(out->unew, unew, sizeof(double) * (size_t)(nf * dim));
        if (out->fs) memcpy(out->fs, fs, sizeof(int64_t) * (size_t)nf);
        out->iters = k;
        out->ratio = ratio;
        out->lambda = lambda;
        out->beta = beta;
        out->converged = ratio < P->tol;
        out->p_ref_used = *p_ref;
        out->umax = umax;
        out->fmax = fmax;
        out->dt_next = dt_next;
    }
    free(coef);
    free(fp);
    free(xk);
    free(vk);
    free(fk);
    free(p0);
    free(rho_all);
    free(u_all);
    free(f);
    free(xs);
    free(us_all);
    free(rhs);
    free(diag);
    free(pk);
    free(pn);
    free(fs);
    free(unew);
    csr_free(&N);
    csr_free(&Nw);
    return 0;
}
