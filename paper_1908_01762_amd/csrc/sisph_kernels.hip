// HIP kernels of the SISPH hot path for gfx950.
//
// One thread per particle in cell order; neighbour lists are slot-major
// [cap][n] so a wavefront of 64 consecutive particles reads each slot with
// one coalesced load, and the gathered neighbour data are mostly L2 hits
// because neighbours sit in nearby cells, i.e. nearby indices.  Workgroups
// are remapped so that each XCD owns one contiguous range of particles
// (its own L2 then holds that range's neighbourhood).  Sums run in the
// template type R (double, or float in the mixed mode); per-particle results,
// the PPE residual and positions are FP64.
//
// Equations are those of Muta, Ramachandran & Negi, arXiv:1908.01762.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "sisph_internal.h"

namespace sisph {

namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t xcd = b % kXcd, idx = b / kXcd, per = G / kXcd, rem = G % kXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

__device__ __forceinline__ int64_t gid_xcd() { return xcd_block() * kBlock + threadIdx.x; }

inline int64_t nblocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

struct Pos {
    const double *c[3];
};
struct PosW {
    double *c[3];
};

inline Pos mkpos(const double *const p[3]) { return Pos{{p[0], p[1], p[2]}}; }
inline PosW mkposw(double *const p[3]) { return PosW{{p[0], p[1], p[2]}}; }

__device__ __forceinline__ double min_image(double v, const Grid &g, int k) {
    if (g.per[k]) {
        if (v > g.Lh[k]) v -= g.L[k];
        else if (v < -g.Lh[k]) v += g.L[k];
    }
    return v;
}

// |d|^2 in exactly the operations of the CPU reference: products rounded,
// then summed left to right, no fused multiply-add.
template <int D>
__device__ __forceinline__ double exact_r2(const double d[3]) {
#pragma clang fp contract(off)
    double s = d[0] * d[0] + d[1] * d[1];
    if (D == 3) s = s + d[2] * d[2];
    return s;
}

__device__ __forceinline__ double wrap_periodic(double x, const Grid &g, int k) {
    if (!g.per[k]) return x;
    if (x >= g.hi[k]) x -= g.L[k];
    else if (x < g.lo[k]) {
        x += g.L[k];
        if (x >= g.hi[k]) x = g.lo[k];
    }
    return x;
}

__device__ __forceinline__ int cell_coord(double x, const Grid &g, int k) {
    double q = floor((x - g.lo[k]) / g.edge[k]);
    int c = q < 0.0 ? 0 : (q > (double)(g.nc[k] - 1) ? g.nc[k] - 1 : (int)q);
    return c;
}

// Stencil cells per axis: c-1, c, c+1, wrapped on periodic axes, skipped
// outside the grid otherwise, each cell at most once.
struct Stencil {
    int v[3][3];
    int n[3];
};

template <int D>
__device__ __forceinline__ void make_stencil(const Grid &g, const int ci[3], Stencil &st) {
    for (int k = 0; k < 3; ++k) {
        st.n[k] = 1;
        st.v[k][0] = 0;
    }
    for (int k = 0; k < D; ++k) {
        int n = 0;
        for (int o = -1; o <= 1; ++o) {
            int c = ci[k] + o;
            if (g.per[k]) c = (c + g.nc[k]) % g.nc[k];
            else if (c < 0 || c >= g.nc[k]) continue;
            bool dup = false;
            for (int t = 0; t < n; ++t) dup |= (st.v[k][t] == c);
            if (!dup) st.v[k][n++] = c;
        }
        st.n[k] = n;
    }
}

// ----------------------------------------------------------- SPH kernels
// Quintic spline: W = s [(3-q)^5 - 6(2-q)^5 + 15(1-q)^5], brackets clipped
// at 0; s = 7/(478 pi h^2) (2D), 1/(120 pi h^3) (3D).
// Wendland C2: W = s (1-q/2)^4 (2q+1), q < 2; s = 7/(4 pi h^2), 21/(16 pi h^3).
template <int KER, int D, typename R>
struct Kern {
    R sig, inv_h;
    __device__ Kern(double h) {
        double s;
        if (KER == SISPH_QUINTIC) s = D == 2 ? 7.0 / (478.0 * kPi * h * h) : 1.0 / (120.0 * kPi * h * h * h);
        else s = D == 2 ? 7.0 / (4.0 * kPi * h * h) : 21.0 / (16.0 * kPi * h * h * h);
        sig = (R)s;
        inv_h = (R)(1.0 / h);
    }
    __device__ __forceinline__ R w(R r) const {
        R q = r * inv_h;
        if (KER == SISPH_QUINTIC) {
            R a = R(3) - q, b = R(2) - q, c = R(1) - q, s = R(0);
            if (a > R(0)) { R a2 = a * a; s += a2 * a2 * a; }
            if (b > R(0)) { R b2 = b * b; s -= R(6) * b2 * b2 * b; }
            if (c > R(0)) { R c2 = c * c; s += R(15) * c2 * c2 * c; }
            return sig * s;
        } else {
            if (q >= R(2)) return R(0);
            R a = R(1) - R(0.5) * q, a2 = a * a;
            return sig * a2 * a2 * (R(2) * q + R(1));
        }
    }
    // (dW/dr) / r: grad_i W_ij = dwr * r_ij; 0 at r = 0.
    __device__ __forceinline__ R dwr(R r) const {
        R q = r * inv_h;
        if (KER == SISPH_QUINTIC) {
            if (r <= R(0)) return R(0);
            R a = R(3) - q, b = R(2) - q, c = R(1) - q, s = R(0);
            if (a > R(0)) { R a2 = a * a; s -= R(5) * a2 * a2; }
            if (b > R(0)) { R b2 = b * b; s += R(30) * b2 * b2; }
            if (c > R(0)) { R c2 = c * c; s -= R(75) * c2 * c2; }
            return sig * inv_h * s / r;
        } else {
            if (q >= R(2)) return R(0);
            R a = R(1) - R(0.5) * q;
            return R(-5) * sig * inv_h * inv_h * a * a * a;
        }
    }
};

// Pair difference r_i - r_j (FP64, minimum image) converted to R.
template <int D, typename R>
__device__ __forceinline__ void pair_diff(const Grid &g, const double xi[3], const Pos &x, int64_t j,
                                          R d[3], R &r2) {
    r2 = R(0);
    for (int k = 0; k < 3; ++k) d[k] = R(0);
    for (int k = 0; k < D; ++k) {
        double v = min_image(xi[k] - x.c[k][j], g, k);
        d[k] = (R)v;
        r2 += d[k] * d[k];
    }
}

// --------------------------------------------------------------- utilities
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_iota(int32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}
__global__ void k_reset_control(Control *c, int what) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (what & RESET_PPE) {
            c->iter = 0;
            c->done = 0;
            c->nonfinite = 0;
            c->ticket = 0;
            c->ratio = 0.0;
            c->num = 0.0;
            c->den = 0.0;
            c->lambda_bits = 0ull;
            c->pmax_key = 0ull;
        }
        if (what & RESET_NEIGHBOURS) {
            c->overflow = 0;
            c->maxcnt = 0;
        }
        if (what & RESET_PREF) {
            c->p_ref_set = 0;
            c->p_ref = 0.0;
        }
    }
}

// atomicMax that skips the atomic when a (possibly stale) read of the
// monotonically growing target already covers v: most threads then issue a
// plain load instead of contending on one address.
__device__ __forceinline__ void max_if_larger(int32_t *t, int32_t v) {
    if (v > __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(t, v);
}
__device__ __forceinline__ void max_if_larger(unsigned long long *t, unsigned long long v) {
    if (v > __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(t, v);
}

// ----------------------------------------------------------------- binning
template <int D>
__global__ void k_bin_keys(Grid g, Pos x, int64_t base, int64_t n, uint32_t *count, uint32_t *key,
                           uint32_t *rank) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int c[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) c[k] = cell_coord(x.c[k][base + i], g, k);
    uint32_t cell = (uint32_t)(((int64_t)c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0]);
    key[i] = cell;
    rank[i] = atomicAdd(&count[cell], 1u);
}

constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

// Exclusive scan of one tile per workgroup; writes the tile total.
__global__ void k_scan_tiles(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tile_sum) {
    __shared__ uint32_t sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
    for (int t = 0; t < kScanItems; ++t) {
        v[t] = (base + t < n) ? in[base + t] : 0u;
        s += v[t];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {   // Hillis-Steele inclusive scan
        uint32_t a = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += a;
        __syncthreads();
    }
    uint32_t run = sh[threadIdx.x] - s;
    for (int t = 0; t < kScanItems; ++t) {
        if (base + t < n) out[base + t] = run;
        run += v[t];
    }
    if (threadIdx.x == kBlock - 1) tile_sum[blockIdx.x] = sh[kBlock - 1];
}

// Exclusive scan of the tile totals by one workgroup (any count); writes the
// grand total to *total.
__global__ void k_scan_sums(uint32_t *tile_sum, int64_t ntiles, uint32_t *total) {
    __shared__ uint32_t sh[kBlock];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < ntiles; b0 += kBlock) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < ntiles ? tile_sum[i] : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            uint32_t a = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < ntiles) tile_sum[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(uint32_t *out, int64_t n, const uint32_t *tile_sum) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] += tile_sum[i / kScanTile];
}

__global__ void k_scatter(const uint32_t *key, const uint32_t *rank, const uint32_t *start, int64_t n,
                          int32_t *perm) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) perm[start[key[i]] + rank[i]] = (int32_t)i;
}

// Orders each cell's slots by sortkey[src] (or by src itself), which makes
// the counting sort's result independent of the atomic ranks.
__global__ void k_cell_sort(const uint32_t *start, int64_t ncell, int32_t *perm, const int32_t *sortkey) {
    int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    uint32_t a = start[c], b = start[c + 1];
    for (uint32_t t = a + 1; t < b; ++t) {
        int32_t v = perm[t];
        int32_t kv = sortkey ? sortkey[v] : v;
        uint32_t u = t;
        while (u > a) {
            int32_t w = perm[u - 1];
            int32_t kw = sortkey ? sortkey[w] : w;
            if (kw <= kv) break;
            perm[u] = w;
            --u;
        }
        perm[u] = v;
    }
}

constexpr int kMaxReorder = 16;
struct ArrList {
    double *a[kMaxReorder];
};

__global__ void k_gather_f64(const int32_t *perm, int64_t n, ArrList src, int narr, double *tmp) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t s = perm[i];
    for (int k = 0; k < narr; ++k) tmp[(int64_t)k * n + i] = src.a[k][s];
}
__global__ void k_copyback_f64(int64_t n, ArrList dst, int narr, const double *tmp) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < narr; ++k) dst.a[k][i] = tmp[(int64_t)k * n + i];
}
__global__ void k_gather_i32(const int32_t *perm, int64_t n, const int32_t *src, int32_t *tmp) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) tmp[i] = src[perm[i]];
}
__global__ void k_copy_i32(int64_t n, int32_t *dst, const int32_t *src) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// -------------------------------------------------------- neighbour lists
// Fluid rows: self in slot 0, then every fluid and wall particle j != i of
// the stencil cells with |r_ij|^2 < R^2 (exact FP64 predicate), in stencil
// order (z, y, x) and, within a cell, in slot order.
template <int D>
__global__ void k_build_fluid(Params P, Pos x, const int32_t *items, const uint32_t *fstart,
                              const uint32_t *wstart, int32_t *nbr, int32_t *cnt, Control *ctl) {
    const int64_t i = gid_xcd();
    if (i >= P.nf) return;
    const Grid &g = P.grid;
    const int64_t nf = P.nf;
    double xi[3] = {0, 0, 0};
    int ci[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) {
        xi[k] = x.c[k][i];
        ci[k] = cell_coord(xi[k], g, k);
    }
    Stencil st;
    make_stencil<D>(g, ci, st);
    int c = 1;
    const int cap = P.cap;
    nbr[i] = (int32_t)i;
    for (int a = 0; a < st.n[2]; ++a)
        for (int b = 0; b < st.n[1]; ++b)
            for (int e = 0; e < st.n[0]; ++e) {
                int64_t cell = ((int64_t)st.v[2][a] * g.nc[1] + st.v[1][b]) * g.nc[0] + st.v[0][e];
                for (int pass = 0; pass < 2; ++pass) {
                    const uint32_t *start = pass == 0 ? fstart : wstart;
                    uint32_t t0 = start[cell], t1 = start[cell + 1];
                    for (uint32_t t = t0; t < t1; ++t) {
                        int64_t j = pass == 0 ? (items ? (int64_t)items[t] : (int64_t)t) : nf + (int64_t)t;
                        if (j == i) continue;
                        double d[3] = {0, 0, 0};
                        for (int k = 0; k < D; ++k) d[k] = min_image(xi[k] - x.c[k][j], g, k);
                        if (exact_r2<D>(d) < P.R2) {
                            if (c < cap) nbr[(int64_t)c * nf + i] = (int32_t)j;
                            ++c;
                        }
                    }
                }
            }
    if (c > cap) {
        atomicOr(&ctl->overflow, 1);
        atomicMax(&ctl->maxcnt, c);
    }
    cnt[i] = c < cap ? c : cap;
}

// Wall rows: fluid particles only, no self.
template <int D>
__global__ void k_build_wall(Params P, Pos x, const int32_t *items, const uint32_t *fstart, int32_t *nbr,
                             int32_t *cnt, Control *ctl) {
    const int64_t w = gid_xcd();
    if (w >= P.nw) return;
    const Grid &g = P.grid;
    const int64_t iw = P.nf + w, nw = P.nw;
    double xi[3] = {0, 0, 0};
    int ci[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) {
        xi[k] = x.c[k][iw];
        ci[k] = cell_coord(xi[k], g, k);
    }
    Stencil st;
    make_stencil<D>(g, ci, st);
    int c = 0;
    const int cap = P.cap;
    for (int a = 0; a < st.n[2]; ++a)
        for (int b = 0; b < st.n[1]; ++b)
            for (int e = 0; e < st.n[0]; ++e) {
                int64_t cell = ((int64_t)st.v[2][a] * g.nc[1] + st.v[1][b]) * g.nc[0] + st.v[0][e];
                for (uint32_t t = fstart[cell]; t < fstart[cell + 1]; ++t) {
                    int64_t j = items ? (int64_t)items[t] : (int64_t)t;
                    double d[3] = {0, 0, 0};
                    for (int k = 0; k < D; ++k) d[k] = min_image(xi[k] - x.c[k][j], g, k);
                    if (exact_r2<D>(d) < P.R2) {
                        if (c < cap) nbr[(int64_t)c * nw + w] = (int32_t)j;
                        ++c;
                    }
                }
            }
    if (c > cap) {
        atomicOr(&ctl->overflow, 1);
        atomicMax(&ctl->maxcnt, c);
    }
    cnt[w] = c < cap ? c : cap;
}

// ------------------------------------------------------------ wall normals
// Section 3.4.1: n*_w = -sum_j (m_j/rho0) grad_w W_wj over wall neighbours,
// zeroed below 1/(4h), else made unit; then n_w = sum_j (m_j/rho0) n*_j W_wj,
// made unit.  Computed once (static walls) straight from the wall cells.
template <int KER, int D>
__global__ void k_wall_normals(Params P, Pos x, const double *m, const uint32_t *wstart, PosW nstar,
                               PosW out, int pass) {
    const int64_t w = gid_xcd();
    if (w >= P.nw) return;
    const Grid &g = P.grid;
    const int64_t nf = P.nf, iw = nf + w;
    Kern<KER, D, double> K(P.h);
    double xi[3] = {0, 0, 0};
    int ci[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) {
        xi[k] = x.c[k][iw];
        ci[k] = cell_coord(xi[k], g, k);
    }
    Stencil st;
    make_stencil<D>(g, ci, st);
    double a[3] = {0, 0, 0};
    for (int aa = 0; aa < st.n[2]; ++aa)
        for (int b = 0; b < st.n[1]; ++b)
            for (int e = 0; e < st.n[0]; ++e) {
                int64_t cell = ((int64_t)st.v[2][aa] * g.nc[1] + st.v[1][b]) * g.nc[0] + st.v[0][e];
                for (uint32_t t = wstart[cell]; t < wstart[cell + 1]; ++t) {
                    int64_t j = nf + t;
                    double d[3] = {0, 0, 0};
                    for (int k = 0; k < D; ++k) d[k] = min_image(xi[k] - x.c[k][j], g, k);
                    double r2 = exact_r2<D>(d);
                    if (!(r2 < P.R2)) continue;
                    double r = sqrt(r2), V = m[j] / P.rho0;
                    if (pass == 0) {
                        double f = K.dwr(r);
                        for (int k = 0; k < D; ++k) a[k] -= V * f * d[k];
                    } else {
                        double W = K.w(r);
                        for (int k = 0; k < D; ++k) a[k] += V * nstar.c[k][t] * W;
                    }
                }
            }
    double mag2 = 0.0;
    for (int k = 0; k < D; ++k) mag2 += a[k] * a[k];
    double mag = sqrt(mag2);
    for (int k = 0; k < D; ++k) {
        double v;
        if (pass == 0) v = mag < 1.0 / (4.0 * P.h) ? 0.0 : a[k] / mag;
        else v = mag > 1e-9 ? a[k] / mag : 0.0;   // cancellation residue: no direction
        out.c[k][w] = v;
    }
}

// ----------------------------------------------------- summation density
// eq. summation_density over fluid + wall neighbours; free-surface flag
// rho_i / rho0 < fs_ratio when free_surface is on (section 3).
template <int KER, int D, typename R>
__global__ void k_density(Params P, Pos x, const double *m, const int32_t *nbr, const int32_t *cnt,
                          double *rho, int32_t *fs) {
    const int64_t i = gid_xcd();
    if (i >= P.nf) return;
    Kern<KER, D, R> K(P.h);
    double xi[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xi[k] = x.c[k][i];
    const int c = cnt[i];
    R s = (R)m[i] * K.w(R(0));
    for (int k = 1; k < c; ++k) {
        int64_t j = nbr[(int64_t)k * P.nf + i];
        R d[3], r2;
        pair_diff<D, R>(P.grid, xi, x, j, d, r2);
        s += (R)m[j] * K.w(sqrt(r2));
    }
    double rh = (double)s;
    rho[i] = rh;
    fs[i] = (P.free_surface && rh / P.rho0 < P.fs_ratio) ? 1 : 0;
}

// ---------------------------------------------------------- wall velocity
// eq. vf: Shepard average of the fluid velocity with a kernel of smoothing
// length h/2; eq. vg-adami: no-slip ghost 2 u_wall - avg, or the slip form
// avg (used for u*); eq. vg-no-normal: any part into the solid is removed.
template <int KER, int D, typename R>
__global__ void k_wall_velocity(Params P, Pos x, Pos uf, PosW uw, Pos wallu, Pos nrm, const int32_t *wnbr,
                                const int32_t *wcnt, int slip) {
    const int64_t w = gid_xcd();
    if (w >= P.nw) return;
    const int64_t iw = P.nf + w;
    Kern<KER, D, R> K(0.5 * P.h);
    double xi[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xi[k] = x.c[k][iw];
    R num[3] = {0, 0, 0}, den = R(0);
    const int c = wcnt[w];
    for (int k = 0; k < c; ++k) {
        int64_t f = wnbr[(int64_t)k * P.nw + w];
        R d[3], r2;
        pair_diff<D, R>(P.grid, xi, x, f, d, r2);
        R W = K.w(sqrt(r2));
        for (int a = 0; a < D; ++a) num[a] += (R)uf.c[a][f] * W;
        den += W;
    }
    double v[3] = {0, 0, 0}, vn = 0.0;
    for (int a = 0; a < D; ++a) {
        double avg = den > R(0) ? (double)num[a] / (double)den : 0.0;
        v[a] = slip ? avg : 2.0 * wallu.c[a][w] - avg;
        vn += v[a] * nrm.c[a][w];
    }
    if (vn < 0.0)
        for (int a = 0; a < D; ++a) v[a] -= vn * nrm.c[a][w];
    for (int a = 0; a < D; ++a) uw.c[a][iw] = v[a];
}

// --------------------------------------------------------------- predictor
// Viscous (eq. mom:sph:visc), artificial viscosity (eq. mom:sph:av, read as
// Monaghan's Pi_ij = -alpha h c_ref mu_ij / rho_bar for u_ij.r_ij < 0,
// force -sum m_j Pi_ij gradW), artificial stress (eq. mom:sph:gtvf:stress:
// sum m_j (A_i/rho_i^2 + A_j/rho_j^2).gradW, A = rho u (x) (u~ - u), A = 0 on
// walls) and gravity; then r* = r^n + dt u~^n (eq. int:rnp1, wrapped) and
// u* = u^n + dt f (eq. int:vint).
template <int KER, int D, typename R>
__global__ void k_predictor(Params P, Pos x, Pos u, Pos ut, const double *m, const double *rho,
                            const int32_t *nbr, const int32_t *cnt, PosW xs, PosW us) {
    const int64_t i = gid_xcd();
    if (i >= P.nf) return;
    Kern<KER, D, R> K(P.h);
    const int64_t nf = P.nf;
    double xi[3] = {0, 0, 0};
    R ui[3] = {0, 0, 0}, si[3] = {0, 0, 0};
    const R rhoi = (R)rho[i];
    for (int k = 0; k < D; ++k) {
        xi[k] = x.c[k][i];
        ui[k] = (R)u.c[k][i];
        si[k] = (R)(ut.c[k][i] - u.c[k][i]);   // u~ - u
    }
    // A_i / rho_i^2 = (u_i / rho_i) (x) (u~_i - u_i)
    const R inv_rhoi = R(1) / rhoi;
    const R eps = (R)P.eps_h, nu4 = (R)(4.0 * P.nu), avc = (R)(P.alpha * P.h * P.c_ref);
    R fv[3] = {0, 0, 0}, fa[3] = {0, 0, 0}, fsr[3] = {0, 0, 0};
    const int c = cnt[i];
    for (int k = 1; k < c; ++k) {
        int64_t j = nbr[(int64_t)k * nf + i];
        R d[3], r2;
        pair_diff<D, R>(P.grid, xi, x, j, d, r2);
        R r = sqrt(r2);
        R dw = K.dwr(r);
        R gw[3];
        for (int a = 0; a < 3; ++a) gw[a] = dw * d[a];
        R F = dw * r2;
        R mj = (R)m[j], rhoj = (R)rho[j];
        R uij[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) uij[a] = ui[a] - (R)u.c[a][j];
        R inv_den = R(1) / (r2 + eps);
        R cv = mj * nu4 / (rhoi + rhoj) * F * inv_den;
        for (int a = 0; a < D; ++a) fv[a] += cv * uij[a];
        R vr = R(0);
        for (int a = 0; a < D; ++a) vr += uij[a] * d[a];
        if (vr < R(0)) {
            R mu = vr * inv_den;
            R Pi = -avc * mu / (R(0.5) * (rhoi + rhoj));
            for (int a = 0; a < D; ++a) fa[a] -= mj * Pi * gw[a];
        }
        // artificial stress: sum_b (A_i/rho_i^2 + A_j/rho_j^2)_ab gw_b
        R sgi = R(0);
        for (int b = 0; b < D; ++b) sgi += si[b] * gw[b];
        R sgj = R(0), uj_over[3] = {0, 0, 0};
        if (j < nf) {
            R inv_rhoj = R(1) / rhoj;
            for (int b = 0; b < D; ++b) {
                R ujb = (R)u.c[b][j];
                sgj += ((R)ut.c[b][j] - ujb) * gw[b];
                uj_over[b] = ujb * inv_rhoj;
            }
        }
        for (int a = 0; a < D; ++a) fsr[a] += mj * (ui[a] * inv_rhoi * sgi + uj_over[a] * sgj);
    }
    const double dt = P.dt;
    for (int a = 0; a < D; ++a) {
        double f = (double)(fv[a] + fa[a] + fsr[a]) + P.g[a];
        double xn;
        {
#pragma clang fp contract(off)
            xn = xi[a] + dt * ut.c[a][i];
        }
        xs.c[a][i] = wrap_periodic(xn, P.grid, a);
        us.c[a][i] = u.c[a][i] + dt * f;
    }
}

// ------------------------------------------------------- wave reductions
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Cached pair of the mixed-precision sweep: neighbour index and FP32 c_ij
// in one 8-byte word, slot-major [cap][nf] like the neighbour lists.
struct PairF {
    int32_t j;
    float c;
};
template <typename R>
struct CoefSlot;
template <>
struct CoefSlot<float> {
    using T = PairF;
};
template <>
struct CoefSlot<double> {
    using T = double;
};

// ------------------------------------------------- PPE RHS and coefficients
// eq. sph-ppe / coeff / coeff1 at r*: RHS_i = sum -m_j/(rho_j dt) u*_ij.gradW,
// c_ij = 4 m_j / (rho_i (rho_i + rho_j)) (r_ij.gradW) / (r^2 + eta h^2),
// D_ii = sum_j c_ij (r^2 + eta h^2, not "+ eta^2").  c_ij is stored in list
// order for the sweeps (with its neighbour index in the mixed mode);
// Lambda = max |RHS/D| over non-free-surface rows (wave max, then one
// atomic per wavefront).
template <int KER, int D, typename R>
__global__ void k_rhs_coef(Params P, Pos xs, Pos us, const double *m, const double *rho, const int32_t *fs,
                           const int32_t *nbr, const int32_t *cnt, typename CoefSlot<R>::T *coef, double *rhs,
                           double *dii, Control *ctl) {
    const int64_t i = gid_xcd();
    const int64_t nf = P.nf;
    unsigned long long lam = 0ull;
    if (i < nf) {
        Kern<KER, D, R> K(P.h);
        double xi[3] = {0, 0, 0};
        R usi[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) {
            xi[k] = xs.c[k][i];
            usi[k] = (R)us.c[k][i];
        }
        const R rhoi = (R)rho[i], eps = (R)P.eps_h, inv_dt = (R)(1.0 / P.dt);
        R s = R(0), Dg = R(0);
        const int c = cnt[i];
        for (int k = 1; k < c; ++k) {
            int64_t j = nbr[(int64_t)k * nf + i];
            R d[3], r2;
            pair_diff<D, R>(P.grid, xi, xs, j, d, r2);
            R dw = K.dwr(sqrt(r2));
            R mj = (R)m[j], rhoj = (R)rho[j];
            R dot = R(0);
            for (int a = 0; a < D; ++a) dot += (usi[a] - (R)us.c[a][j]) * d[a];
            s -= mj / rhoj * inv_dt * dw * dot;
            R cij = R(4) * mj / (rhoi * (rhoi + rhoj)) * (dw * r2) / (r2 + eps);
            if constexpr (sizeof(R) == 4) coef[(int64_t)k * nf + i] = PairF{(int32_t)j, cij};
            else coef[(int64_t)k * nf + i] = cij;
            Dg += cij;
        }
        double rr = (double)s, dd = (double)Dg;
        rhs[i] = rr;
        dii[i] = dd;
        if (dd != 0.0 && !fs[i]) lam = (unsigned long long)__double_as_longlong(fabs(rr / dd));
    }
    lam = wave_max_u64(lam);   // non-negative doubles order like their bits
    if ((threadIdx.x & 63) == 0 && lam) max_if_larger(&ctl->lambda_bits, lam);
}

// ------------------------------------------------------- block reductions
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sums (a, b) over the workgroup; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double &a, double &b) {
    __shared__ double sh[2][kBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0.0;
        b = 0.0;
        for (int t = 0; t < kBlock / 64; ++t) {
            a += sh[0][t];
            b += sh[1][t];
        }
    }
}

// Stopping rule of eq. convergence after L sweeps, from the per-workgroup
// partial sums of sweep L-1.  Every workgroup of the next launch sums the
// same partials in the same order, so all reach the same decision without
// any cross-workgroup synchronisation (the kernel boundary makes the
// partials visible).  The partials are loaded into registers before the
// workgroup's own row work (kPartialRegs per thread and array when they fit)
// so their latency overlaps it; stopped_after() then reduces and decides.
// Workgroup 0 records the result.
constexpr int kPartialRegs = 8;

struct PartialLoad {
    double a[kPartialRegs], b[kPartialRegs];
};

__device__ __forceinline__ void load_partials(const double *partial, int64_t nblk, int L, PartialLoad &pl) {
    const double *pa = partial + (int64_t)((L - 1) & 1) * 2 * nblk;
#pragma unroll
    for (int t = 0; t < kPartialRegs; ++t) {
        const int64_t k = threadIdx.x + (int64_t)t * kBlock;
        pl.a[t] = k < nblk ? pa[k] : 0.0;
        pl.b[t] = k < nblk ? pa[nblk + k] : 0.0;
    }
}

__device__ bool stopped_after(const Params &P, const double *partial, int64_t nblk, int L, const PartialLoad &pl,
                              int done0, double lam, Control *ctl) {
    __shared__ double sh[2][kBlock / 64];
    __shared__ int stop_sh;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int t = 0; t < kPartialRegs; ++t) {
        a += pl.a[t];
        b += pl.b[t];
    }
    if (nblk > (int64_t)kPartialRegs * kBlock) {   // large grids: the rest, in order
        const double *pa = partial + (int64_t)((L - 1) & 1) * 2 * nblk;
        for (int64_t k = threadIdx.x + (int64_t)kPartialRegs * kBlock; k < nblk; k += kBlock) {
            a += pa[k];
            b += pa[nblk + k];
        }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0 && done0) {
        stop_sh = 1;   // sticky: an earlier launch stopped the solve
    } else if (threadIdx.x == 0) {
        a = 0.0;
        b = 0.0;
        for (int t = 0; t < kBlock / 64; ++t) {
            a += sh[0][t];
            b += sh[1][t];
        }
        if (P.conv_norm == SISPH_CONV_MEAN) lam *= (double)P.nf;
        const double scale = lam > b ? lam : b;
        const double ratio = scale > 0.0 ? a / scale : (a > 0.0 ? INFINITY : 0.0);
        const bool bad = !isfinite(a) || !isfinite(b);
        bool stop;
        if (P.forced_iters > 0) stop = L >= P.forced_iters;
        else stop = (L >= P.min_iter && ratio < P.tol) || L >= P.max_iter;
        stop = stop || bad;
        stop_sh = stop ? 1 : 0;
        if (blockIdx.x == 0) {
            ctl->num = a;
            ctl->den = b;
            ctl->ratio = ratio;
            if (bad) ctl->nonfinite = 1;
            if (stop) {
                ctl->iter = L;
                ctl->done = 1;
            }
        }
    }
    __syncthreads();
    return stop_sh != 0;
}

// ------------------------------------------------------------- PPE sweep
// eq. p-sor with omega: p_i^{k+1} = w (RHS_i + sum_j c_ij p_j^k) / D_ii
// + (1 - w) p_i^k; p = 0 where D_ii = 0 or on free-surface rows (section 3).
// Double-buffered (Jacobi): reads iterate k, writes k+1.  The neighbour sum
// is taken in batches of kSweepBatch slots whose loads are all issued
// before the first is used (the sum still runs in slot order).  Mixed: the
// cached (j, c_ij) words and the FP32 copy of iterate k; FP64: indices,
// FP64 coefficients and iterate k.
// First batch: slots 1..kSweepFirst loaded without waiting for the row's
// count (every slot below cap is inside the list storage; slots past the
// count hold stale words and are discarded by the select), so the row loads,
// these loads and the partial-sum loads form one round trip.  Longer rows
// continue in batches of kSweepBatch.
constexpr int kSweepFirst = 24;
constexpr int kSweepBatch = 8;

template <typename R, int NB>
__device__ __forceinline__ void load_batch(int64_t i, int64_t nf, int k0, int c, int cap, bool blind,
                                           const typename CoefSlot<R>::T *coef, const int32_t *nbr,
                                           int32_t (&jj)[NB], R (&cc)[NB]) {
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int k = k0 + t;
        int ks = blind ? (k < cap ? k : cap - 1) : (k < c ? k : c - 1);
        const int64_t at = (int64_t)ks * nf + i;
        int32_t j;
        R cf;
        if constexpr (sizeof(R) == 4) {
            const PairF w = coef[at];
            j = w.j;
            cf = w.c;
        } else {
            j = nbr[at];
            cf = coef[at];
        }
        jj[t] = j;
        cc[t] = cf;
    }
}

template <typename R, int NB>
__device__ __forceinline__ R gather_sum(int64_t i, int k0, int c, const int32_t (&jj)[NB], const R (&cc)[NB],
                                        const double *pc, const float *qc, R s) {
    R pv[NB];
    int32_t js[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) js[t] = (k0 + t < c) ? jj[t] : (int32_t)i;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        if constexpr (sizeof(R) == 4) pv[t] = qc[js[t]];
        else pv[t] = pc[js[t]];
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) s += ((k0 + t < c) ? cc[t] : R(0)) * pv[t];
    return s;
}

template <typename R>
__global__ void k_ppe_sweep(Params P, int L, double *p0, double *p1, float *q0, float *q1,
                            const typename CoefSlot<R>::T *coef, const int32_t *nbr, const int32_t *cnt,
                            const double *rhs, const double *dii, const int32_t *fs, double *partial,
                            Control *ctl) {
    // L = sweeps completed before this launch (the host counts launches).
    // Whether the solve has already stopped is decided per workgroup behind
    // a barrier (stopped_after), never per wavefront.
    const int64_t nblk = gridDim.x;
    // control values the decision needs, loaded up front: done (set by an
    // earlier launch, or by workgroup 0 of this one from the same partials,
    // which gives the same answer) and Lambda (fixed during the solve)
    const int done0 = __hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double lam = __longlong_as_double((long long)ctl->lambda_bits);
    PartialLoad pl;
    if (L > 0) load_partials(partial, nblk, L, pl);
    const double *pc = (L & 1) ? p1 : p0;
    double *pn = (L & 1) ? p0 : p1;
    const float *qc = (L & 1) ? q1 : q0;
    float *qn = (L & 1) ? q0 : q1;
    const int64_t blk = xcd_block();
    const int64_t i = blk * kBlock + threadIdx.x;
    const int64_t nf = P.nf;
    double v = 0.0, pold = 0.0;
    if (i < nf) {
        // one round trip: row values, the first batch of (j, c) words and
        // (above) the partial sums
        int32_t jj[kSweepFirst];
        R cc[kSweepFirst];
        load_batch<R, kSweepFirst>(i, nf, 1, 0, P.cap, true, coef, nbr, jj, cc);
        const double D = dii[i], r = rhs[i];
        const int32_t f = fs[i], c = cnt[i];
        pold = pc[i];
        R s = gather_sum<R, kSweepFirst>(i, 1, c, jj, cc, pc, qc, R(0));
        for (int k0 = 1 + kSweepFirst; k0 < c; k0 += kSweepBatch) {
            int32_t jb[kSweepBatch];
            R cb[kSweepBatch];
            load_batch<R, kSweepBatch>(i, nf, k0, c, P.cap, false, coef, nbr, jb, cb);
            s = gather_sum<R, kSweepBatch>(i, k0, c, jb, cb, pc, qc, s);
        }
        if (D != 0.0 && !f) v = P.omega * (r + (double)s) / D + (1.0 - P.omega) * pold;
    }
    // the decision for L sweeps gates every write of this launch
    if (L > 0 && stopped_after(P, partial, nblk, L, pl, done0, lam, ctl)) return;
    double a = 0.0, b = 0.0;
    if (i < nf) {
        pn[i] = v;
        if constexpr (sizeof(R) == 4) qn[i] = (float)v;
        a = fabs(v - pold);
        b = fabs(v);
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        double *pw = partial + (int64_t)(L & 1) * 2 * nblk;
        pw[blk] = a;
        pw[nblk + blk] = b;
        if (blk == 0) ctl->iter = L + 1;
    }
}

// eq. p-shepard: p_w = [sum_f p_f W_wf + (g - a_w) . sum_f rho_f r_wf W_wf]
// / sum_f W_wf over fluid neighbours (static wall: a_w = 0); 0 without
// neighbours; clamped at 0 on free-surface problems.  Writes the wall slots
// of the iterate the next sweep reads.
template <int KER, int D, typename R>
__global__ void k_wall_pressure(Params P, int L, Pos xs, double *p0, double *p1, float *q0, float *q1,
                                const double *rho, const int32_t *wnbr, const int32_t *wcnt, Control *ctl,
                                int force) {
    // L: sweeps completed (the iterate the next sweep reads); with force the
    // final count recorded in the control block is used instead
    if (!force && ctl->done) return;
    const int iter = force ? ctl->iter : L;
    double *pc = (iter & 1) ? p1 : p0;
    float *qc = (iter & 1) ? q1 : q0;
    const int64_t w = gid_xcd();
    if (w >= P.nw) return;
    const int64_t iw = P.nf + w;
    Kern<KER, D, R> K(P.h);
    double xi[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xi[k] = xs.c[k][iw];
    R sp = R(0), sr[3] = {0, 0, 0}, sw = R(0);
    const int c = wcnt[w];
    for (int k = 0; k < c; ++k) {
        int64_t f = wnbr[(int64_t)k * P.nw + w];
        R d[3], r2;
        pair_diff<D, R>(P.grid, xi, xs, f, d, r2);
        R W = K.w(sqrt(r2));
        R pf = sizeof(R) == 4 ? (R)qc[f] : (R)pc[f];
        sp += pf * W;
        R rw = (R)rho[f] * W;
        for (int a = 0; a < D; ++a) sr[a] += rw * d[a];
        sw += W;
    }
    double pw = 0.0;
    if (sw > R(0)) {
        double gs = 0.0;
        for (int a = 0; a < D; ++a) gs += P.g[a] * (double)sr[a];
        pw = ((double)sp + gs) / (double)sw;
    }
    if (P.free_surface && pw < 0.0) pw = 0.0;
    pc[iw] = pw;
    qc[iw] = (float)pw;
}

__device__ __forceinline__ unsigned long long order_key(double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_val(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

__global__ void k_pmax(Params P, const double *p, Control *ctl) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long k = i < P.nf ? order_key(p[i]) : 0ull;
    k = wave_max_u64(k);
    if ((threadIdx.x & 63) == 0 && k) max_if_larger(&ctl->pmax_key, k);
}
// p_ref for internal flows: twice the largest pressure after the first
// solve, then held (section 2.1).
__global__ void k_pref_finish(Control *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && !ctl->p_ref_set) {
        ctl->p_ref = 2.0 * order_val(ctl->pmax_key);
        ctl->p_ref_set = 1;
    }
}

__global__ void k_copy_p32(const double *p, float *q, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) q[i] = (float)p[i];
}

// ----------------------------------------------- pressure force, correction
// eq. mom:sph:press:pij (asymm) or mom:sph:press:symm, then
// u^{n+1} = u* + dt f_p (eq. int:vnp1).
template <int KER, int D, typename R>
__global__ void k_correct(Params P, Pos xs, Pos us, const double *m, const double *rho, const double *p,
                          const int32_t *nbr, const int32_t *cnt, PosW un) {
    const int64_t i = gid_xcd();
    if (i >= P.nf) return;
    Kern<KER, D, R> K(P.h);
    const int64_t nf = P.nf;
    double xi[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xi[k] = xs.c[k][i];
    const double pi = p[i], rhoi_d = rho[i];
    const R rhoi = (R)rhoi_d, pi_r = (R)(pi / (rhoi_d * rhoi_d));
    R f[3] = {0, 0, 0};
    const int c = cnt[i];
    const bool symm = P.pgrad == SISPH_SYMM;
    for (int k = 1; k < c; ++k) {
        int64_t j = nbr[(int64_t)k * nf + i];
        R d[3], r2;
        pair_diff<D, R>(P.grid, xi, xs, j, d, r2);
        R dw = K.dwr(sqrt(r2));
        R mj = (R)m[j];
        double rhoj = rho[j];
        R cf;
        if (symm) cf = -mj * (pi_r + (R)(p[j] / (rhoj * rhoj)));
        else cf = -mj / (rhoi * (R)rhoj) * (R)(p[j] - pi);
        cf *= dw;
        for (int a = 0; a < D; ++a) f[a] += cf * d[a];
    }
    for (int a = 0; a < D; ++a) un.c[a][i] = us.c[a][i] + P.dt * (double)f[a];
}

// --------------------------------------------------------- GTVF sub-steps
// f = -p0_i sum_j m_j / rho_j^2 grad_i W(r_ij^{k-1}, h~) on the frozen r*
// neighbour lists (eq. mom:sph:gtvf), walls fixed;
// r^k = r^{k-1} + dtau u~^{k-1} + dtau^2/2 f, u~^k = u~^{k-1} + dtau f
// (eqs. int:gtvf:pos, int:gtvf:vel:tmp), no wrap inside the sub-steps.
template <int KER, int D, typename R>
__global__ void k_gtvf(Params P, Pos xsrc, PosW xdst, PosW vk, int first, const double *m, const double *rho,
                       const double *p, const int32_t *nbr, const int32_t *cnt, const Control *ctl) {
    const int64_t i = gid_xcd();
    if (i >= P.nf) return;
    const bool ext = P.gtvf == SISPH_GTVF_EXTERNAL;
    Kern<KER, D, R> K(ext ? 0.5 * P.h : P.h);
    const int64_t nf = P.nf;
    double xi[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xi[k] = xsrc.c[k][i];
    const double pref = ctl->p_ref;
    double p0 = pref;
    if (ext) {
        double a = 10.0 * fabs(p[i]);
        p0 = a < pref ? a : pref;
    }
    R s[3] = {0, 0, 0};
    const int c = cnt[i];
    for (int k = 1; k < c; ++k) {
        int64_t j = nbr[(int64_t)k * nf + i];
        R d[3], r2;
        pair_diff<D, R>(P.grid, xi, xsrc, j, d, r2);
        R dw = K.dwr(sqrt(r2));
        R rhoj = (R)rho[j];
        R cf = (R)m[j] / (rhoj * rhoj) * dw;
        for (int a = 0; a < D; ++a) s[a] += cf * d[a];
    }
    const double dtau = P.dt / (double)P.gtvf_K;
    for (int a = 0; a < D; ++a) {
        double f = -p0 * (double)s[a];
        double v = first ? 0.0 : vk.c[a][i];
        xdst.c[a][i] = xi[a] + dtau * v + 0.5 * dtau * dtau * f;
        vk.c[a][i] = v + dtau * f;
    }
}

// u~^{n+1} = u^{n+1} + (r^K - r^0)/dt (eq. int:vhatnp2);
// r^{n+1} = r^n + dt/2 (u~^{n+1} + u~^n) (eq. int:rnp2), wrapped.
template <int D>
__global__ void k_advance(Params P, PosW x, PosW u, PosW ut, Pos un, Pos xs, Pos xk) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= P.nf) return;
    for (int a = 0; a < D; ++a) {
        double utn = un.c[a][i] + (xk.c[a][i] - xs.c[a][i]) / P.dt;
        double xn = x.c[a][i] + 0.5 * P.dt * (utn + ut.c[a][i]);
        x.c[a][i] = wrap_periodic(xn, P.grid, a);
        ut.c[a][i] = utn;
        u.c[a][i] = un.c[a][i];
    }
}

}  // namespace

// ===================================================================== host
#define SISPH_DISPATCH_D(P, CALL)      \
    do {                               \
        if ((P).dim == 2) {            \
            constexpr int D = 2;       \
            CALL;                      \
        } else {                       \
            constexpr int D = 3;       \
            CALL;                      \
        }                              \
    } while (0)

#define SISPH_DISPATCH_KDR(P, CALL)                                        \
    do {                                                                   \
        if ((P).precision == SISPH_MIXED) {                                \
            using R = float;                                               \
            if ((P).kernel == SISPH_QUINTIC) {                             \
                constexpr int KER = SISPH_QUINTIC;                         \
                SISPH_DISPATCH_D(P, CALL);                                 \
            } else {                                                       \
                constexpr int KER = SISPH_WENDLAND_C2;                     \
                SISPH_DISPATCH_D(P, CALL);                                 \
            }                                                              \
        } else {                                                           \
            using R = double;                                              \
            if ((P).kernel == SISPH_QUINTIC) {                             \
                constexpr int KER = SISPH_QUINTIC;                         \
                SISPH_DISPATCH_D(P, CALL);                                 \
            } else {                                                       \
                constexpr int KER = SISPH_WENDLAND_C2;                     \
                SISPH_DISPATCH_D(P, CALL);                                 \
            }                                                              \
        }                                                                  \
    } while (0)

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill_u32<<<nblocks(n), kBlock, 0, s>>>(p, v, n);
}
void fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill_f64<<<nblocks(n), kBlock, 0, s>>>(p, v, n);
}
void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n > 0) k_iota<<<nblocks(n), kBlock, 0, s>>>(p, n);
}
void reset_control(Control *c, int what, hipStream_t s) { k_reset_control<<<1, 64, 0, s>>>(c, what); }

void bin_particles(const Params &P, const double *const pos[3], int64_t base, int64_t n, const int32_t *sortkey,
                   State &S, uint32_t *start, int32_t *perm, hipStream_t s) {
    const int64_t nc = P.grid.ncell;
    fill_u32(S.count, 0u, nc, s);
    if (n > 0) SISPH_DISPATCH_D(P, (k_bin_keys<D><<<nblocks(n), kBlock, 0, s>>>(P.grid, mkpos(pos), base, n,
                                                                               S.count, S.key, S.rank)));
    const int64_t ntiles = (nc + kScanTile - 1) / kScanTile;
    k_scan_tiles<<<ntiles, kBlock, 0, s>>>(S.count, start, nc, S.scan_tmp);
    k_scan_sums<<<1, kBlock, 0, s>>>(S.scan_tmp, ntiles, start + nc);
    k_scan_add<<<nblocks(nc), kBlock, 0, s>>>(start, nc, S.scan_tmp);
    if (n > 0) {
        k_scatter<<<nblocks(n), kBlock, 0, s>>>(S.key, S.rank, start, n, perm);
        k_cell_sort<<<nblocks(nc), kBlock, 0, s>>>(start, nc, perm, sortkey);
    }
}

void reorder_f64(const int32_t *perm, int64_t n, double *const *arrays, int narr, double *tmp, hipStream_t s) {
    if (n <= 0) return;
    for (int a0 = 0; a0 < narr; a0 += kMaxReorder) {
        ArrList L{};
        int k = 0;
        for (; k < kMaxReorder && a0 + k < narr; ++k) L.a[k] = arrays[a0 + k];
        k_gather_f64<<<nblocks(n), kBlock, 0, s>>>(perm, n, L, k, tmp);
        k_copyback_f64<<<nblocks(n), kBlock, 0, s>>>(n, L, k, tmp);
    }
}

void reorder_i32(const int32_t *perm, int64_t n, int32_t *a, int32_t *tmp, hipStream_t s) {
    if (n <= 0) return;
    k_gather_i32<<<nblocks(n), kBlock, 0, s>>>(perm, n, a, tmp);
    k_copy_i32<<<nblocks(n), kBlock, 0, s>>>(n, a, tmp);
}

void build_neighbors(const Params &P, const double *const pos[3], State &S, hipStream_t s) {
    SISPH_DISPATCH_D(P, (k_build_fluid<D><<<nblocks(P.nf), kBlock, 0, s>>>(P, mkpos(pos), S.items, S.fstart,
                                                                          S.wstart, S.nbr, S.cnt, S.ctl)));
    if (P.nw > 0)
        SISPH_DISPATCH_D(P, (k_build_wall<D><<<nblocks(P.nw), kBlock, 0, s>>>(P, mkpos(pos), S.items, S.fstart,
                                                                             S.wnbr, S.wcnt, S.ctl)));
}

void wall_normals(const Params &P, State &S, hipStream_t s) {
    if (P.nw <= 0) return;
    double *ns[3] = {S.tmp, S.tmp + P.nw, S.tmp + 2 * P.nw};
    SISPH_DISPATCH_KDR(P, (k_wall_normals<KER, D><<<nblocks(P.nw), kBlock, 0, s>>>(
                              P, mkpos(S.x), S.m, S.wstart, mkposw(ns), mkposw(ns), 0)));
    SISPH_DISPATCH_KDR(P, (k_wall_normals<KER, D><<<nblocks(P.nw), kBlock, 0, s>>>(
                              P, mkpos(S.x), S.m, S.wstart, mkposw(ns), mkposw(S.nrm), 1)));
}

void density(const Params &P, State &S, hipStream_t s) {
    SISPH_DISPATCH_KDR(P, (k_density<KER, D, R><<<nblocks(P.nf), kBlock, 0, s>>>(P, mkpos(S.x), S.m, S.nbr,
                                                                                  S.cnt, S.rho, S.fs)));
}

void wall_velocity(const Params &P, const double *const pos[3], const double *const uf[3],
                   double *const uw[3], int slip, State &S, hipStream_t s) {
    if (P.nw <= 0) return;
    SISPH_DISPATCH_KDR(P, (k_wall_velocity<KER, D, R><<<nblocks(P.nw), kBlock, 0, s>>>(
                              P, mkpos(pos), mkpos(uf), mkposw(uw), mkpos(S.wallu), mkpos(S.nrm), S.wnbr,
                              S.wcnt, slip)));
}

void predictor(const Params &P, State &S, hipStream_t s) {
    SISPH_DISPATCH_KDR(P, (k_predictor<KER, D, R><<<nblocks(P.nf), kBlock, 0, s>>>(
                              P, mkpos(S.x), mkpos(S.u), mkpos(S.ut), S.m, S.rho, S.nbr, S.cnt, mkposw(S.xs),
                              mkposw(S.us))));
}

void rhs_coef(const Params &P, State &S, hipStream_t s) {
    SISPH_DISPATCH_KDR(P, (k_rhs_coef<KER, D, R><<<nblocks(P.nf), kBlock, 0, s>>>(
                              P, mkpos(S.xs), mkpos(S.us), S.m, S.rho, S.fs, S.nbr, S.cnt,
                              (typename CoefSlot<R>::T *)S.coef, S.rhs,
                              S.dii, S.ctl)));
}

void ppe_iteration(const Params &P, State &S, int L, hipStream_t s) {
    float *q0 = S.p32, *q1 = S.p32 + P.ntot;
    if (P.nw > 0)
        SISPH_DISPATCH_KDR(P, (k_wall_pressure<KER, D, R><<<nblocks(P.nw), kBlock, 0, s>>>(
                                  P, L, mkpos(S.xs), S.p[0], S.p[1], q0, q1, S.rho, S.wnbr, S.wcnt, S.ctl, 0)));
    if (P.precision == SISPH_MIXED)
        k_ppe_sweep<float><<<S.nblk_f, kBlock, 0, s>>>(P, L, S.p[0], S.p[1], q0, q1, (const PairF *)S.coef, S.nbr,
                                                      S.cnt, S.rhs, S.dii, S.fs, S.partial, S.ctl);
    else
        k_ppe_sweep<double><<<S.nblk_f, kBlock, 0, s>>>(P, L, S.p[0], S.p[1], q0, q1, (const double *)S.coef,
                                                       S.nbr, S.cnt, S.rhs, S.dii, S.fs, S.partial, S.ctl);
}

void wall_pressure_final(const Params &P, State &S, hipStream_t s) {
    if (P.nw <= 0) return;
    float *q0 = S.p32, *q1 = S.p32 + P.ntot;
    SISPH_DISPATCH_KDR(P, (k_wall_pressure<KER, D, R><<<nblocks(P.nw), kBlock, 0, s>>>(
                              P, 0, mkpos(S.xs), S.p[0], S.p[1], q0, q1, S.rho, S.wnbr, S.wcnt, S.ctl, 1)));
}

void pressure_max(const Params &P, State &S, int final_parity, hipStream_t s) {
    k_pmax<<<nblocks(P.nf), kBlock, 0, s>>>(P, S.p[final_parity], S.ctl);
    k_pref_finish<<<1, 64, 0, s>>>(S.ctl);
}

void copy_p32(const Params &P, State &S, hipStream_t s) {
    k_copy_p32<<<nblocks(P.ntot), kBlock, 0, s>>>(S.p[0], S.p32, P.ntot);
}

void correct(const Params &P, State &S, int final_parity, hipStream_t s) {
    SISPH_DISPATCH_KDR(P, (k_correct<KER, D, R><<<nblocks(P.nf), kBlock, 0, s>>>(
                              P, mkpos(S.xs), mkpos(S.us), S.m, S.rho, S.p[final_parity], S.nbr, S.cnt,
                              mkposw(S.un))));
}

void gtvf_substep(const Params &P, State &S, int final_parity, int k, hipStream_t s) {
    const double *const *src = k == 0 ? (const double *const *)S.xs : (const double *const *)S.xk[(k - 1) & 1];
    SISPH_DISPATCH_KDR(P, (k_gtvf<KER, D, R><<<nblocks(P.nf), kBlock, 0, s>>>(
                              P, mkpos(src), mkposw(S.xk[k & 1]), mkposw(S.vk), k == 0 ? 1 : 0, S.m, S.rho,
                              S.p[final_parity], S.nbr, S.cnt, S.ctl)));
}

void advance(const Params &P, State &S, int kfinal, hipStream_t s) {
    const double *const *xk = kfinal < 0 ? (const double *const *)S.xs : (const double *const *)S.xk[kfinal & 1];
    SISPH_DISPATCH_D(P, (k_advance<D><<<nblocks(P.nf), kBlock, 0, s>>>(P, mkposw(S.x), mkposw(S.u), mkposw(S.ut),
                                                                      mkpos(S.un), mkpos(S.xs), mkpos(xk))));
}

}  // namespace sisph
