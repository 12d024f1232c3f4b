// HIP kernels of the SISPH hot path for gfx950.
//
// One thread per particle in cell order; neighbour lists are slot-major
// [cap][n] so a wavefront of 64 consecutive particles reads each slot with
// one coalesced load, and the gathered neighbour data are mostly cache hits
// because neighbours sit in nearby cells, i.e. nearby indices.  Workgroups
// are remapped so that each XCD owns one contiguous range of particles (its
// own L2 then holds that range's neighbourhood).  Sums run in the template
// type R (double, or float in the mixed mode); per-particle results, the PPE
// residual and positions are FP64.
//
// Every kernel is a body run(P, S, blk, nblk, c, ...) for one case's
// workgroup blk of nblk, with two wrappers: one case (parameters by value)
// or a batch of cases (one launch; each workgroup finds its case in a
// device table).  Results do not depend on the wrapper.
//
// Equations are those of Muta, Ramachandran & Negi, arXiv:1908.01762.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <type_traits>

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

inline int64_t nblocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

struct Pos {
    const double *c[3];
};
struct PosW {
    double *c[3];
};

__device__ __forceinline__ Pos mkpos(double *const p[3]) { return Pos{{p[0], p[1], p[2]}}; }
__device__ __forceinline__ PosW mkposw(double *const p[3]) { return PosW{{p[0], p[1], p[2]}}; }

__device__ __forceinline__ double min_image(double v, const Grid &g, int k) {
    if (g.per[k]) {
        if (v > g.Lh[k]) v -= g.L[k];
        else if (v < -g.Lh[k]) v += g.L[k];
    }
    return v;
}

// The same without branches (both shifted values formed, one selected), for
// loops that load several operands before using any; PER false: no
// direction is periodic.
template <bool PER>
__device__ __forceinline__ double min_image_sel(double v, const Grid &g, int k) {
    if constexpr (!PER) {
        return v;
    } else {
        const double lo = v + g.L[k], hi = v - g.L[k];
        const double w = v > g.Lh[k] ? hi : (v < -g.Lh[k] ? lo : v);
        return g.per[k] ? w : v;
    }
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
// The 3^D cell stencil of a cell: per dimension the cells at offsets -1, 0,
// +1 (wrapped on periodic axes), in that order, in fixed slots; a slot is
// off when it falls outside a non-periodic grid or repeats an earlier slot
// (a periodic axis of fewer than three cells).  Dimensions beyond D hold
// cell 0 in slot 0 only.  Loops over the slots unroll, so the struct stays
// in registers.
struct Stencil {
    int v[3][3];
    bool ok[3][3];
};

template <int D>
__device__ __forceinline__ void make_stencil(const Grid &g, const int ci[3], Stencil &st) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            st.v[k][s] = 0;
            st.ok[k][s] = s == 0;
        }
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            int c = ci[k] + s - 1;
            bool ok = true;
            if (g.per[k]) c = (c + g.nc[k]) % g.nc[k];
            else ok = c >= 0 && c < g.nc[k];
#pragma unroll
            for (int t = 0; t < s; ++t) ok = ok && !(st.ok[k][t] && st.v[k][t] == c);
            st.v[k][s] = c;
            st.ok[k][s] = ok;
        }
}

// arr[idx] for idx < 3 by selects (no dynamically indexed local array)
template <typename T>
__device__ __forceinline__ T pick3(const T (&arr)[3], int idx) {
    return idx == 0 ? arr[0] : (idx == 1 ? arr[1] : arr[2]);
}

__device__ __forceinline__ int64_t stencil_cell(const Grid &g, const Stencil &st, int a, int b, int e) {
    return ((int64_t)st.v[2][a] * g.nc[1] + st.v[1][b]) * g.nc[0] + st.v[0][e];
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

// Pair difference r_i - r_j (FP64, minimum image) converted to R, from the
// gathered position of j.
template <int D, typename R>
__device__ __forceinline__ void pair_diff_v(const Grid &g, const double xi[3], const double xj[3], R d[3],
                                            R &r2) {
    r2 = R(0);
    for (int k = 0; k < 3; ++k) d[k] = R(0);
    for (int k = 0; k < D; ++k) {
        double v = min_image(xi[k] - xj[k], g, k);
        d[k] = (R)v;
        r2 += d[k] * d[k];
    }
}

template <int D, typename R>
__device__ __forceinline__ void pair_diff(const Grid &g, const double xi[3], const Pos &x, int64_t j,
                                          R d[3], R &r2) {
    double xj[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xj[k] = x.c[k][j];
    pair_diff_v<D, R>(g, xi, xj, d, r2);
}

// Pair loops take the neighbour list kPairBatch slots at a time: the
// batch's indices, then every field its pair terms read, are loaded before
// any term is formed, so a wavefront keeps kPairBatch x fields gathers in
// flight instead of a chain of dependent round trips per pair.  Slots at or
// past the row's count load the fallback row (a valid index) and add
// nothing; the terms are added in slot order, as one slot at a time would.
constexpr int kPairBatch = 4;

// Indices of slots k0 .. k0+kPairBatch-1 of a slot-major list [cap][rows].
__device__ __forceinline__ void batch_slots(const int32_t *list, int64_t rows, int64_t row, int k0, int c,
                                            int cap, int64_t fallback, int64_t (&jb)[kPairBatch]) {
#pragma unroll
    for (int t = 0; t < kPairBatch; ++t) {
        const int k = k0 + t < cap ? k0 + t : cap - 1;
        const int32_t j = list[(int64_t)k * rows + row];
        jb[t] = k0 + t < c ? (int64_t)j : fallback;
    }
}

template <int D>
__device__ __forceinline__ void batch_pos(const Pos &x, const int64_t (&jb)[kPairBatch], double (&xj)[kPairBatch][3]) {
#pragma unroll
    for (int t = 0; t < kPairBatch; ++t) {
        for (int k = 0; k < 3; ++k) xj[t][k] = 0.0;
        for (int k = 0; k < D; ++k) xj[t][k] = x.c[k][jb[t]];
    }
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// atomicMax that skips the atomic when a (possibly stale) read of the
// monotonically growing target already covers v.
__device__ __forceinline__ void max_if_larger(unsigned long long *t, unsigned long long v) {
    if (v > __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(t, v);
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

// FP32 counterparts for the plain FP32 mode.
__device__ __forceinline__ float wave_sum_f(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ void block_sum2_f(float &a, float &b) {
    __shared__ float sh[2][kBlock / 64];
    a = wave_sum_f(a);
    b = wave_sum_f(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0.f;
        b = 0.f;
        for (int t = 0; t < kBlock / 64; ++t) {
            a += sh[0][t];
            b += sh[1][t];
        }
    }
}

// A per-particle result in the case's precision: rounded to FP32 in the
// plain FP32 mode, kept otherwise.
__device__ __forceinline__ bool plain32(const Params &P) { return P.precision == SISPH_FP32; }
__device__ __forceinline__ double rp(const Params &P, double v) { return plain32(P) ? (double)(float)v : v; }

__device__ __forceinline__ unsigned long long order_key(double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_val(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// ================================================================ wrappers
// XCD: logical workgroup = XCD-contiguous remap of the hardware index (the
// default), or the hardware index itself.  Either way each logical
// workgroup does the same work, so results do not depend on it.
template <bool XCD>
__device__ __forceinline__ int64_t logical_block() {
    if constexpr (XCD) return xcd_block();
    else return (int64_t)blockIdx.x;
}

template <class F, bool XCD, class... A>
__global__ __launch_bounds__(kBlock) void k_one(const Params P, const State S, A... a) {
    F::run(P, S, logical_block<XCD>(), (int64_t)gridDim.x, 0, a...);
}

template <class F, int KIND, bool XCD, class... A>
__global__ __launch_bounds__(kBlock) void k_many(const CaseEntry *__restrict__ tab,
                                                 const int32_t *__restrict__ owner,
                                                 const int64_t *__restrict__ first, A... a) {
    const int64_t b = logical_block<XCD>();
    const int c = owner[b];
    const CaseEntry &e = tab[c];
    F::run(e.P, e.S, b - first[c], e.nblk[KIND], c, a...);
}

template <class F, int KIND, bool XCD = true, class... A>
void launch(const Target &T, A... a) {
    if (!T.batched) {
        const int64_t nb = kind_blocks(*T.P, KIND);
        if (nb > 0) k_one<F, XCD, A...><<<nb, kBlock, 0, T.s>>>(*T.P, *T.S, a...);
    } else if (T.total[KIND] > 0) {
        k_many<F, KIND, XCD, A...><<<T.total[KIND], kBlock, 0, T.s>>>(T.tab, T.owner[KIND], T.first[KIND], a...);
    }
}

#define ROW int64_t i = blk * kBlock + threadIdx.x

// ================================================================== bodies
// ----------------------------------------------------------------- control
struct ResetControl {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t, int64_t, int, int what) {
        if (what & RESET_PPE)   // the persistent solve's barrier words
            for (int k = threadIdx.x; k < kSyncWords; k += kBlock) S.sync[k] = 0u;
        if (threadIdx.x != 0) return;
        Control *c = S.ctl;
        if (what & RESET_DT) {
            c->dt = P.dt;
            c->dt_next = P.dt;
        }
        if (what & RESET_STEP) {
            c->dt = c->dt_next;
            c->umax2_bits = 0ull;
            c->fmax2_bits = 0ull;
            c->g_full = 0;
            c->g_disp_bits = 0ull;
        }
        if (what & RESET_PPE) {
            c->barrier_late = 0;
            c->iter = 0;
            c->done = 0;
            c->stopped_at = INT32_MAX;
            c->nonfinite = 0;
            c->ratio = 0.0;
            c->num = 0.0;
            c->den = 0.0;
            c->lambda_bits = 0ull;
            c->pmax_key = 0ull;
            c->bicg_brk = 0;
            c->wide = 0;
            for (int k = 0; k < 2; ++k) {
                c->bicg_rho[k] = 1.0;
                c->bicg_alpha[k] = 1.0;
                c->bicg_omega[k] = 1.0;
            }
        }
        if (what & RESET_NEIGHBOURS) {
            c->overflow = 0;
            c->maxcnt = 0;
            c->pk_overflow = 0;
        }
        if (what & RESET_PREF) {
            c->p_ref_set = 0;
            c->p_ref = 0.0;
        }
    }
};

struct GatherControl {
    static __device__ __forceinline__ void run(const Params &, const State &S, int64_t, int64_t, int c, Control *out) {
        if (threadIdx.x == 0) out[c] = *S.ctl;
    }
};

// ----------------------------------------------------------------- binning
// Counting sort: count per cell (atomic rank), exclusive scan of the
// counts, scatter, then each cell's slots ordered by a key (the particle's
// original index, or its current slot), which makes the result independent
// of the atomic ranks.
struct ZeroCount {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i < P.grid.ncell) S.count[i] = 0u;
    }
};

template <int D>
struct BinKeys {
    // walls: rows [nf, nf+nw) at r^n; fluid: rows [0, nf) at r^n or r*
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int which, int walls) {
        ROW;
        const int64_t n = walls ? P.nw : P.nf, base = walls ? P.nf : 0;
        if (i >= n) return;
        double *const *pos = which == POS_XS ? S.xs : S.x;
        int c[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) c[k] = cell_coord(pos[k][base + i], P.grid, k);
        const uint32_t cell = (uint32_t)(((int64_t)c[2] * P.grid.nc[1] + c[1]) * P.grid.nc[0] + c[0]);
        S.key[i] = cell;
        // One atomic per distinct cell of the wavefront (its lanes are mostly
        // in a few cells: the particles are in the last binning's order), the
        // lanes of a cell ranked by lane order after the cell's base.  Ranks
        // still depend on the order atomics arrive in; CellSort fixes the
        // order within each cell.
        const uint64_t lane_lt = (1ull << (threadIdx.x & 63)) - 1ull;
        uint64_t todo = __ballot(1);
        while (todo) {
            const int lead = __ffsll((unsigned long long)todo) - 1;
            const uint32_t key = __shfl(cell, lead, 64);
            const uint64_t same = __ballot(cell == key) & todo;
            uint32_t first = 0u;
            if ((int)(threadIdx.x & 63) == lead) first = atomicAdd(&S.count[key], (uint32_t)__popcll(same));
            first = __shfl(first, lead, 64);
            if (cell == key) S.rank[i] = first + (uint32_t)__popcll(same & lane_lt);
            todo &= ~same;
        }
    }
};

// Exclusive scan of one tile of counts per workgroup; writes the tile total.
struct ScanTiles {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int walls) {
        __shared__ uint32_t sh[kBlock];
        uint32_t *out = walls ? S.wstart : S.fstart;
        const int64_t n = P.grid.ncell;
        const int64_t base = blk * kScanTile + threadIdx.x * kScanItems;
        uint32_t v[kScanItems], s = 0;
        for (int t = 0; t < kScanItems; ++t) {
            v[t] = (base + t < n) ? S.count[base + t] : 0u;
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
        if (threadIdx.x == kBlock - 1) S.scan_tmp[blk] = sh[kBlock - 1];
    }
};

// Exclusive scan of the tile totals by one workgroup; writes the grand
// total to start[ncell].
struct ScanSums {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t, int64_t, int, int walls) {
        __shared__ uint32_t sh[kBlock];
        __shared__ uint32_t carry;
        uint32_t *out = walls ? S.wstart : S.fstart;
        const int64_t ntiles = (P.grid.ncell + kScanTile - 1) / kScanTile;
        if (threadIdx.x == 0) carry = 0;
        __syncthreads();
        for (int64_t b0 = 0; b0 < ntiles; b0 += kBlock) {
            const int64_t i = b0 + threadIdx.x;
            const uint32_t v = i < ntiles ? S.scan_tmp[i] : 0u;
            sh[threadIdx.x] = v;
            __syncthreads();
            for (int off = 1; off < kBlock; off <<= 1) {
                uint32_t a = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
                __syncthreads();
                sh[threadIdx.x] += a;
                __syncthreads();
            }
            if (i < ntiles) S.scan_tmp[i] = carry + sh[threadIdx.x] - v;
            __syncthreads();
            if (threadIdx.x == 0) carry += sh[kBlock - 1];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[P.grid.ncell] = carry;
    }
};

struct ScanAdd {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int walls) {
        ROW;
        uint32_t *out = walls ? S.wstart : S.fstart;
        if (i < P.grid.ncell) out[i] += S.scan_tmp[i / kScanTile];
    }
};

struct Scatter {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int walls) {
        ROW;
        const uint32_t *start = walls ? S.wstart : S.fstart;
        if (i < (walls ? P.nw : P.nf)) S.perm[start[S.key[i]] + S.rank[i]] = (int32_t)i;
    }
};

// The particles of each cell in ascending (x, key) order (the atomic ranks
// of BinKeys leave them in arrival order): one order for every later pass
// over a cell, and one in which the neighbour build can skip the far part
// of the cells left and right of a row's own.  x is the first coordinate
// of the positions binned (as an order-preserving integer); the key breaks
// ties.  sortkey: 0 = slot index, 1 = fluid original index, 2 = wall
// original index (keys are unique).  Each half of a wavefront takes one
// cell: a cell of up to 32 particles holds one per lane, and a particle's
// place is the number of the cell's particles that order before it
// (shuffles within the half); a larger cell is sorted by insertion on the
// half's first lane.
struct CellSort {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int walls,
                                               int sortkey, int which) {
        constexpr int G = 64 / kCellsPerWave;   // lanes per cell
        const int64_t cell = blk * (kBlock / G) + threadIdx.x / G;
        const int lane = threadIdx.x % G;
        if (cell >= P.grid.ncell) return;   // the whole group
        const uint32_t *start = walls ? S.wstart : S.fstart;
        const int32_t *key = sortkey == 1 ? S.id : (sortkey == 2 ? S.wid : nullptr);
        const double *px = (which == POS_XS ? S.xs : S.x)[0] + (walls ? P.nf : 0);
        int32_t *perm = S.perm;
        const uint32_t a = start[cell], n = start[cell + 1] - a;
        if (n < 2) return;
        if (n <= (uint32_t)G) {
            const bool in = lane < (int)n;
            const int32_t v = in ? perm[a + lane] : 0;
            const int32_t kv = in ? (key ? key[v] : v) : INT32_MAX;
            const unsigned long long xv = in ? order_key(px[v]) : ~0ull;
            uint32_t rank = 0;
            for (uint32_t m = 0; m < n; ++m) {
                const unsigned long long xm = __shfl(xv, (int)m, G);
                const int32_t km = __shfl(kv, (int)m, G);
                rank += (xm < xv) || (xm == xv && km < kv);
            }
            if (in) perm[a + rank] = v;   // every lane has read before any writes
            return;
        }
        if (lane != 0) return;
        for (uint32_t t = a + 1; t < a + n; ++t) {
            const int32_t v = perm[t];
            const int32_t kv = key ? key[v] : v;
            const unsigned long long xv = order_key(px[v]);
            uint32_t u = t;
            while (u > a) {
                const int32_t w = perm[u - 1];
                const int32_t kw = key ? key[w] : w;
                const unsigned long long xw = order_key(px[w]);
                if (xw < xv || (xw == xv && kw < kv)) break;
                perm[u] = w;
                --u;
            }
            perm[u] = v;
        }
    }
};

// Reorder of the step-start fluid state (r, u, u~, p, m, original index)
// into the new cell order: gather into scratch, then copy back.
template <int D>
struct ReorderFluid {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int phase) {
        ROW;
        const int64_t n = P.nf;
        if (i >= n) return;
        double *arr[3 * D + 2];
        int k = 0;
        for (int a = 0; a < D; ++a) arr[k++] = S.x[a];
        for (int a = 0; a < D; ++a) arr[k++] = S.u[a];
        for (int a = 0; a < D; ++a) arr[k++] = S.ut[a];
        arr[k++] = S.p[0];
        arr[k++] = S.m;
        int32_t *itmp = (int32_t *)(S.tmp + (int64_t)(3 * D + 2) * n);
        if (phase == 0) {
            const int32_t s = S.perm[i];
            for (int t = 0; t < 3 * D + 2; ++t) S.tmp[(int64_t)t * n + i] = arr[t][s];
            itmp[i] = S.id[s];
        } else {
            for (int t = 0; t < 3 * D + 2; ++t) arr[t][i] = S.tmp[(int64_t)t * n + i];
            S.id[i] = itmp[i];
        }
    }
};

// Reorder of the fluid state into the r* cell order, after the binning at
// r*: during the second stage the neighbour candidates of one stencil row
// (three cells along x) are then one contiguous index range.  Every fluid
// array read later in the step moves through scratch (gathered through the
// r* permutation, then copied back), in two batches that fit the scratch:
// batch 0 r^n, u^n, u~^n, r*, u*; batch 1 p^n, m, rho, m / rho^2, the
// free-surface flag, the original index, the acceleration kept for the
// adaptive step and the FP32 copies of m and rho.
template <int D>
struct ReorderStage2 {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int batch,
                                               int phase) {
        ROW;
        const int64_t n = P.nf;
        if (i >= n) return;
        const int64_t s = phase == 0 ? (int64_t)S.perm[i] : 0;
        int nd = 0;
        auto mvd = [&](double *col) {
            double *t = S.tmp + (int64_t)(nd++) * n;
            if (phase == 0) t[i] = col[s];
            else col[i] = t[i];
        };
        if (batch == 0) {
            for (int a = 0; a < D; ++a) mvd(S.x[a]);
            for (int a = 0; a < D; ++a) mvd(S.u[a]);
            for (int a = 0; a < D; ++a) mvd(S.ut[a]);
            for (int a = 0; a < D; ++a) mvd(S.xs[a]);
            for (int a = 0; a < D; ++a) mvd(S.us[a]);
            return;
        }
        mvd(S.p[0]);
        mvd(S.m);
        mvd(S.rho);
        if (P.adaptive_dt)
            for (int a = 0; a < D; ++a) mvd(S.vk[a]);
        const bool mixed = f32_sums(P.precision);
        if (!mixed) mvd((double *)S.mr2);
        // 4-byte columns after the 8-byte ones
        uint32_t *wt = (uint32_t *)(S.tmp + (int64_t)nd * n);
        int nw = 0;
        auto mvw = [&](void *colv) {
            uint32_t *col = (uint32_t *)colv;
            uint32_t *t = wt + (int64_t)(nw++) * n;
            if (phase == 0) t[i] = col[s];
            else col[i] = t[i];
        };
        mvw(S.fs);
        mvw(S.id);
        if (mixed) {
            mvw(S.mr2);
            mvw(S.m32);
            mvw(S.rho32);
        }
    }
};

template <int D>
struct ReorderWalls {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int phase) {
        ROW;
        const int64_t n = P.nw, nf = P.nf;
        if (i >= n) return;
        double *arr[2 * D + 1];
        int k = 0;
        for (int a = 0; a < D; ++a) arr[k++] = S.x[a] + nf;
        arr[k++] = S.m + nf;
        for (int a = 0; a < D; ++a) arr[k++] = S.wallu[a];
        int32_t *itmp = (int32_t *)(S.tmp + (int64_t)(2 * D + 1) * n);
        if (phase == 0) {
            const int32_t s = S.perm[i];
            for (int t = 0; t < 2 * D + 1; ++t) S.tmp[(int64_t)t * n + i] = arr[t][s];
            itmp[i] = S.wid[s];
        } else {
            for (int t = 0; t < 2 * D + 1; ++t) arr[t][i] = S.tmp[(int64_t)t * n + i];
            S.wid[i] = itmp[i];
        }
    }
};

// -------------------------------------------------------- neighbour lists
// Fluid rows: self in slot 0, then every fluid and wall particle j != i of
// the stencil cells with |r_ij|^2 < R^2 (exact FP64 predicate), in stencil
// order (z, y, x) and, within a cell, fluid then walls, each in slot order.
// At r* as at r^n the fluid is in the cell order of the positions the
// lists are built at (the state is reordered after each binning), so a
// cell's particles are its slot range.
//
// The workgroup's rows (consecutive in cell order) share most stencil
// cells, so for each stencil row (a, b) the workgroup first stages, in LDS,
// the positions and indices of every fluid and wall particle in the cell-id
// range spanned by its rows' cells of that stencil row (one coalesced pass
// instead of one gather per row and candidate).  A cell outside the staged
// range, or a range too large to stage (periodic wrap, clustering), is read
// from global memory as before; the visiting order, hence the lists, are
// the same either way.  1016 candidates: positions, index and (for the
// density) mass in 32 bytes each keep five workgroups per CU in FP32 sums.
constexpr int kStageCap = 1016;

// The summation density (eq. summation_density: m_i W(0) + sum_j m_j W_ij
// over fluid and wall neighbours, in list order, in the working precision)
// formed by the build at r^n as it lists each neighbour: the terms, their
// order and arithmetic of a pass over the finished list, without that
// pass's second gather of every neighbour's position and mass.
// Its arithmetic is written out with no contraction into fused
// multiply-adds: the compiler's choice of where to fuse could otherwise
// differ between the kernel instances (one case, a batch) that inline it.
template <int KER, int D, typename R>
struct DensAcc {
    Kern<KER, D, R> K;
    R s;
    __device__ explicit DensAcc(double h) : K(h), s(R(0)) {}
    __device__ __forceinline__ R w(R r) const {
#pragma clang fp contract(off)
        const R q = r * K.inv_h;
        if (KER == SISPH_QUINTIC) {
            const R a = R(3) - q, b = R(2) - q, c = R(1) - q;
            R t = R(0);
            if (a > R(0)) {
                const R a2 = a * a;
                t = t + a2 * a2 * a;
            }
            if (b > R(0)) {
                const R b2 = b * b;
                t = t - R(6) * b2 * b2 * b;
            }
            if (c > R(0)) {
                const R c2 = c * c;
                t = t + R(15) * c2 * c2 * c;
            }
            return K.sig * t;
        } else {
            if (q >= R(2)) return R(0);
            const R a = R(1) - R(0.5) * q, a2 = a * a;
            return K.sig * a2 * a2 * (R(2) * q + R(1));
        }
    }
    __device__ __forceinline__ void self(R mi) { s = mi * w(R(0)); }
    __device__ __forceinline__ void add(const Grid &g, const double xi[3], const double xj[3], R mj) {
#pragma clang fp contract(off)
        R r2 = R(0);
        for (int k = 0; k < D; ++k) {
            const R d = (R)min_image(xi[k] - xj[k], g, k);
            r2 = r2 + d * d;
        }
        s = s + mj * w(sqrt(r2));
    }
};
// (the build at r*: no density)
struct NoDens {
    float s;
    __device__ explicit NoDens(double) : s(0.0f) {}
};

// The GTVF short list of a row (P.g_sub, at r*): the listed neighbours with
// |r_ij|^2 < g_R2, in list order, without the row itself.
struct ShortList {
    int32_t *slot;   // the next entry (slot-major [g_cap][nf])
    int c;
    bool on;
    __device__ __forceinline__ void add(const Params &P, int32_t j, double r2) {
        if (!on || !(r2 < P.g_R2)) return;
        if (c < P.g_cap) *slot = j;
        slot += P.nf;
        ++c;
    }
};

template <int D, bool DENS, class Acc>
__device__ __forceinline__ void test_cell_global(const Params &P, const State &S, const Pos &x,
                                                 const int32_t *items, int64_t i, const double xi[3],
                                                 int64_t cell, int &c, Acc &da, ShortList &sl) {
    const int64_t nf = P.nf;
    for (int pass = 0; pass < 2; ++pass) {
        const uint32_t *start = pass == 0 ? S.fstart : S.wstart;
        const uint32_t t0 = start[cell], t1 = start[cell + 1];
        for (uint32_t t = t0; t < t1; ++t) {
            const int64_t j = pass == 0 ? (items ? (int64_t)items[t] : (int64_t)t) : nf + (int64_t)t;
            if (j == i) continue;
            double xj[3] = {0, 0, 0}, d[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) {
                xj[k] = x.c[k][j];
                d[k] = min_image(xi[k] - xj[k], P.grid, k);
            }
            const double r2 = exact_r2<D>(d);
            if (r2 < P.R2) {
                if (c < P.cap) S.nbr[(int64_t)c * nf + i] = (int32_t)j;
                ++c;
                if constexpr (DENS) da.add(P.grid, xi, xj, (decltype(da.s))S.m[j]);
                else sl.add(P, (int32_t)j, r2);
            }
        }
    }
}

// Candidates t0 .. t1-1 of the staged copy against row i, kScanBatch at a
// time: the batch's indices and coordinates are read before any is
// tested, so their LDS reads overlap; the set, its order and the counts are
// those of one candidate at a time.
constexpr int kScanBatch = 4;

template <int D, bool PER>
__device__ __forceinline__ bool staged_hit(const Params &P, const Grid &g, const double (*sx)[kStageCap],
                                           const int32_t *sj, uint32_t t, int32_t self, const double xi[3],
                                           int32_t &j, double (&xj)[3], double &r2) {
    j = sj[t];
    for (int k = 0; k < 3; ++k) xj[k] = 0.0;
    for (int k = 0; k < D; ++k) xj[k] = sx[k][t];
    double d[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) d[k] = min_image_sel<PER>(xi[k] - xj[k], g, k);
    r2 = exact_r2<D>(d);
    return (j != self) & (r2 < P.R2);
}

template <int D, bool PER>
__device__ __forceinline__ bool staged_hit(const Params &P, const Grid &g, const double (*sx)[kStageCap],
                                           const int32_t *sj, uint32_t t, int32_t self, const double xi[3],
                                           int32_t &j, double &r2) {
    double xj[3];
    return staged_hit<D, PER>(P, g, sx, sj, t, self, xi, j, xj, r2);
}


// (with DENS, each neighbour's density term is added as it is listed; sm
// holds the staged masses)
template <int D, bool PER, bool DENS, class Acc, typename RM>
__device__ __forceinline__ void scan_staged(const Params &P, const Grid &g, const double (*sx)[kStageCap],
                                            const int32_t *sj, const RM *sm, uint32_t t0, uint32_t t1,
                                            int64_t i, const double xi[3], int32_t *nbr, int &c, Acc &da,
                                            ShortList &sl) {
    constexpr int U = kScanBatch;
    const int64_t nf = P.nf;
    const int32_t self = (int32_t)i;
    // the row's next list slot, moved on by a stride per entry (no index
    // product per entry)
    int32_t *slot = nbr + (int64_t)c * nf + i;
    uint32_t t = t0;
    if constexpr (DENS) {
        for (; t + (U - 1) < t1; t += U) {
            int32_t jv[U];
            bool hv[U];
            double rv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) hv[u] = staged_hit<D, PER>(P, g, sx, sj, t + u, self, xi, jv[u], rv[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (hv[u]) {
                    if (c < P.cap) *slot = jv[u];
                    slot += nf;
                    ++c;
                    // (the position read again from LDS rather than held)
                    double xj[3] = {0, 0, 0};
                    for (int k = 0; k < D; ++k) xj[k] = sx[k][t + u];
                    da.add(g, xi, xj, sm[t + u]);
                }
        }
    } else {
        for (; t + (U - 1) < t1; t += U) {
            int32_t jv[U];
            bool hv[U];
            double rv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) hv[u] = staged_hit<D, PER>(P, g, sx, sj, t + u, self, xi, jv[u], rv[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (hv[u]) {
                    if (c < P.cap) *slot = jv[u];
                    slot += nf;
                    ++c;
                    sl.add(P, jv[u], rv[u]);
                }
        }
    }
    for (; t < t1; ++t) {
        int32_t j;
        double xj[3], r2;
        if (staged_hit<D, PER>(P, g, sx, sj, t, self, xi, j, xj, r2)) {
            if (c < P.cap) *slot = j;
            slot += nf;
            ++c;
            if constexpr (DENS) da.add(g, xi, xj, sm[t]);
            else sl.add(P, j, r2);
        }
    }
}

// Within a cell the particles are in ascending x (CellSort).  For a
// particle j of the cell left of row i's own (x_j <= x_i, the grid not
// periodic along x), fl(x_i - x_j)^2 does not increase with x_j; once it
// reaches R^2 so does the exact |d|^2 (the other rounded squares only add
// to it), so the cell's particles that can be in reach are a suffix: LEFT
// returns its first position in [t0, t1).  For the cell to the right they
// are a prefix, and !LEFT returns its end.  Particles cut off are exactly
// ones the full test rejects, and the rest keep their order.
template <bool LEFT>
__device__ __forceinline__ uint32_t reach_cut(const double *sx0, uint32_t t0, uint32_t t1, double xi0, double R2) {
#pragma clang fp contract(off)
    while (t0 < t1) {
        const uint32_t m = t0 + ((t1 - t0) >> 1);
        const double dx = xi0 - sx0[m];
        const bool far = dx * dx >= R2;
        if (LEFT ? far : !far) t0 = m + 1;
        else t1 = m;
    }
    return t0;
}

// With DENS (the build at r^n) it also forms the summation density and the
// free-surface flag of each row (DensAcc).
template <int KER, int D, typename R, bool DENS>
struct BuildFluid {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int which) {
        __shared__ double sx[3][kStageCap];
        __shared__ int32_t sj[kStageCap];
        __shared__ R sm[DENS ? kStageCap : 1];   // masses (density build only)
        __shared__ long long red_lo[kBlock / 64], red_hi[kBlock / 64];
        __shared__ long long seg[2];
        __shared__ uint32_t rng[4];   // fluid [F0, F1), wall [W0, W1) candidate slots
        ROW;
        const bool live = i < P.nf;
        const Grid &g = P.grid;
        const int64_t nf = P.nf;
        const Pos x = mkpos(which == POS_XS ? S.xs : S.x);
        const int32_t *items = nullptr;   // the fluid is in the cell order of these positions
        const bool periodic = g.per[0] || g.per[1] || g.per[2];
        double xi[3] = {0, 0, 0};
        int ci[3] = {0, 0, 0};
        Stencil st;
        int c = 1;
        typename std::conditional<DENS, DensAcc<KER, D, R>, NoDens>::type da(P.h);
        ShortList sl{nullptr, 0, !DENS && P.g_sub && which == POS_XS && live};
        if (sl.on) sl.slot = S.gnbr + i;
        if (live) {
            for (int k = 0; k < D; ++k) {
                xi[k] = x.c[k][i];
                ci[k] = cell_coord(xi[k], g, k);
            }
            make_stencil<D>(g, ci, st);
            S.nbr[i] = (int32_t)i;
            if constexpr (DENS) da.self((R)S.m[i]);
        }
        constexpr int na = D == 3 ? 3 : 1;
        for (int a = 0; a < na; ++a)
            for (int b = 0; b < 3; ++b) {
                // this stencil row's cells: (va, vb, v[0][e]) for the slots e on
                const bool row_ok = live && pick3(st.ok[2], a) && pick3(st.ok[1], b);
                const int64_t row_base = ((int64_t)pick3(st.v[2], a) * g.nc[1] + pick3(st.v[1], b)) * g.nc[0];
                // the cell-id range of this stencil row over the workgroup
                long long lo = LLONG_MAX, hi = -1;
                if (row_ok)
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        if (!st.ok[0][e]) continue;
                        const long long cc = row_base + st.v[0][e];
                        lo = cc < lo ? cc : lo;
                        hi = cc > hi ? cc : hi;
                    }
                for (int off = 32; off > 0; off >>= 1) {
                    const long long ol = __shfl_xor(lo, off, 64), oh = __shfl_xor(hi, off, 64);
                    lo = ol < lo ? ol : lo;
                    hi = oh > hi ? oh : hi;
                }
                if ((threadIdx.x & 63) == 0) {
                    red_lo[threadIdx.x >> 6] = lo;
                    red_hi[threadIdx.x >> 6] = hi;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    long long l = LLONG_MAX, h = -1;
                    for (int w = 0; w < kBlock / 64; ++w) {
                        l = red_lo[w] < l ? red_lo[w] : l;
                        h = red_hi[w] > h ? red_hi[w] : h;
                    }
                    uint32_t f0 = 0, f1 = 0, w0 = 0, w1 = 0;
                    if (h >= 0) {
                        f0 = S.fstart[l];
                        f1 = S.fstart[h + 1];
                        w0 = S.wstart[l];
                        w1 = S.wstart[h + 1];
                    }
                    const bool fits = h >= 0 && (int64_t)(f1 - f0) + (int64_t)(w1 - w0) <= kStageCap;
                    seg[0] = fits ? l : 1;   // empty range when nothing is staged
                    seg[1] = fits ? h : 0;
                    rng[0] = f0;
                    rng[1] = fits ? f1 : f0;
                    rng[2] = w0;
                    rng[3] = fits ? w1 : w0;
                }
                __syncthreads();
                const long long s_lo = seg[0], s_hi = seg[1];
                const uint32_t F0 = rng[0], nF = rng[1] - rng[0], W0 = rng[2], nW = rng[3] - rng[2];
                for (uint32_t t = threadIdx.x; t < nF + nW; t += kBlock) {
                    const int64_t j = t < nF ? (items ? (int64_t)items[F0 + t] : (int64_t)(F0 + t))
                                             : nf + (int64_t)(W0 + (t - nF));
                    for (int k = 0; k < D; ++k) sx[k][t] = x.c[k][j];
                    sj[t] = (int32_t)j;
                    if constexpr (DENS) sm[t] = (R)S.m[j];
                }
                __syncthreads();
                // Not periodic along x and the row's cells of this stencil
                // row all staged: they are consecutive cells, so their fluid
                // (walls) are one run of the staged copy; the run starts at
                // the first particle of the left cell that can be in reach
                // and ends after the last one of the right cell (see
                // reach_cut), and is scanned in one loop, fluid then walls.
                const int cx = ci[0];
                const int64_t c_first = row_base + (cx > 0 ? cx - 1 : cx);
                const int64_t c_last = row_base + (cx < g.nc[0] - 1 ? cx + 1 : cx);
                const bool flat = row_ok && !g.per[0] && c_first >= s_lo && c_last <= s_hi;
                if (flat)
                    for (int pass = 0; pass < 2; ++pass) {
                        const uint32_t *start = pass == 0 ? S.fstart : S.wstart;
                        const uint32_t base = (pass == 0 ? F0 : W0) - (pass == 0 ? 0u : nF);
                        const int64_t cc = row_base + cx;
                        uint32_t t0 = start[c_first] - base, t1 = start[c_last + 1] - base;
                        if (c_first < cc) t0 = reach_cut<true>(sx[0], t0, start[cc] - base, xi[0], P.R2);
                        if (c_last > cc) t1 = reach_cut<false>(sx[0], start[cc + 1] - base, t1, xi[0], P.R2);
                        if (periodic)
                            scan_staged<D, true, DENS>(P, g, sx, sj, sm, t0, t1, i, xi, S.nbr, c, da, sl);
                        else
                            scan_staged<D, false, DENS>(P, g, sx, sj, sm, t0, t1, i, xi, S.nbr, c, da, sl);
                    }
                else if (row_ok)
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        if (!st.ok[0][e]) continue;
                        const int64_t cell = row_base + st.v[0][e];
                        if (cell < s_lo || cell > s_hi) {
                            test_cell_global<D, DENS>(P, S, x, items, i, xi, cell, c, da, sl);
                            continue;
                        }
                        // fluid then walls of this cell, from the staged copy
                        for (int pass = 0; pass < 2; ++pass) {
                            const uint32_t *start = pass == 0 ? S.fstart : S.wstart;
                            const uint32_t base = pass == 0 ? F0 : W0;
                            const uint32_t shift = pass == 0 ? 0u : nF;
                            const uint32_t t0 = start[cell] - base + shift, t1 = start[cell + 1] - base + shift;
                            if (periodic)
                                scan_staged<D, true, DENS>(P, g, sx, sj, sm, t0, t1, i, xi, S.nbr, c, da, sl);
                            else
                                scan_staged<D, false, DENS>(P, g, sx, sj, sm, t0, t1, i, xi, S.nbr, c, da, sl);
                        }
                    }
                __syncthreads();   // the next stencil row overwrites the staged copy
            }
        if (!live) return;
        if (c > P.cap) {
            atomicOr(&S.ctl->overflow, 1);
            atomicMax(&S.ctl->maxcnt, c);
        }
        S.cnt[i] = c < P.cap ? c : P.cap;
        if (sl.on) {
            if (sl.c > P.g_cap) atomicOr(&S.ctl->g_full, 1);   // the sub-steps take the full lists
            S.gcnt[i] = sl.c < P.g_cap ? sl.c : P.g_cap;
        }
        if constexpr (DENS) {
            // eq. summation_density; free-surface flag rho_i / rho0 <
            // fs_ratio when free_surface is on (section 3)
            const double rh = (double)da.s;
            S.rho[i] = rh;
            const bool low = plain32(P) ? (float)rh / (float)P.rho0 < (float)P.fs_ratio : rh / P.rho0 < P.fs_ratio;
            S.fs[i] = (P.free_surface && low) ? 1 : 0;
        }
    }
};

// Packed codes of the lists at r* (walled Jacobi cases on grids periodic in
// no direction), one pass after the build.  First each workgroup's staging
// record: its rows are in cell order, so their cells are one id range
// [cf, cl]; for each stencil row (dy, dz) the cells [cf, cl] shifted by it
// and widened by one along x are one cell-id interval, whose fluid
// particles are one index interval, and so are its wall particles.  The
// 2 NR intervals, one after the other, are what the workgroup's sweep
// copies into LDS; it is staged when they fit in kStageBytes of iterate
// values.  Then each list entry j of a staged workgroup's rows becomes its
// position in that copy: the interval of the row's own stencil row that
// holds j (the row's three cells lie in it) and the offset into it.  The
// row's range of stencil row r starts at the cell start of its first cell;
// the ranges of a row are in ascending order and a list visits them in
// that order, so the range of j is the last one starting at or below j.
// Lists and codes are read and written coalesced (the build's stores are
// scattered: each row finds its neighbours at its own pace).  A workgroup
// that is not staged keeps no codes; its sweeps read the lists.
__device__ __forceinline__ void put12(uint32_t (&w)[3], int f, uint32_t code) {
    const int b = 12 * f, k = b >> 5, o = b & 31;
    w[k] |= code << o;
    if (o > 20) w[k + 1] |= code >> (32 - o);
}

template <int D>
struct PackCodes {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        if (!P.packed) return;   // (batched: the other cases of the group)
        constexpr int NR = D == 3 ? 9 : 3, NQ = 2 * NR;
        __shared__ int64_t span[2];
        __shared__ int32_t sb[NQ], sp[NQ + 1];
        __shared__ int32_t staged;
        const int64_t nf = P.nf, r0 = blk * kBlock;
        const int64_t r1 = (r0 + kBlock < nf ? r0 + kBlock : nf) - 1;
        const Grid &g = P.grid;
        const Pos x = mkpos(S.xs);
        if (threadIdx.x < 2) {
            const int64_t rr = threadIdx.x == 0 ? r0 : r1;
            int cc[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) cc[k] = cell_coord(x.c[k][rr], g, k);
            span[threadIdx.x] = ((int64_t)cc[2] * g.nc[1] + cc[1]) * g.nc[0] + cc[0];
        }
        __syncthreads();
        if (threadIdx.x < NQ) {
            const int r = (int)threadIdx.x % NR;
            const bool wall = (int)threadIdx.x >= NR;
            const int64_t dz = D == 3 ? r / 3 - 1 : 0, dy = D == 3 ? r % 3 - 1 : r - 1;
            const int64_t off = (dz * (int64_t)g.nc[1] + dy) * (int64_t)g.nc[0];
            int64_t lo = span[0] + off - 1, hi = span[1] + off + 1;
            lo = lo < 0 ? 0 : lo;
            hi = hi > g.ncell - 1 ? g.ncell - 1 : hi;
            int64_t b = 0, n = 0;
            if (lo <= hi) {
                const uint32_t *st = wall ? S.wstart : S.fstart;
                b = (int64_t)st[lo];
                n = (int64_t)st[hi + 1] - b;
                if (wall) b += nf;
            }
            sb[threadIdx.x] = (int32_t)b;
            sp[threadIdx.x + 1] = (int32_t)n;
        }
        __syncthreads();
        int32_t *rec = S.stagerec + blk * kStageRec;
        if (threadIdx.x == 0) {
            sp[0] = 0;
            for (int e = 1; e <= NQ; ++e) sp[e] += sp[e - 1];
            const bool periodic = g.per[0] || g.per[1] || g.per[2];
            const int cap = kStageBytes / (f32_sums(P.precision) ? 4 : 8);
            staged = !periodic && sp[NQ] <= cap;
            if (!staged) atomicAdd(&S.ctl->pk_overflow, 1);
            rec[0] = staged;
        }
        __syncthreads();
        if (threadIdx.x < NQ) rec[1 + threadIdx.x] = sb[threadIdx.x];
        if (threadIdx.x <= NQ) rec[1 + NQ + threadIdx.x] = sp[threadIdx.x];
        ROW;
        if (!staged || i >= nf) return;
        int ci[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) ci[k] = cell_coord(x.c[k][i], g, k);
        Stencil st;
        make_stencil<D>(g, ci, st);
        constexpr int na = D == 3 ? 3 : 1;
        int64_t fs[NR], ws[NR];
        int e0 = 0;
        while (e0 < 2 && !pick3(st.ok[0], e0)) ++e0;
        const int x0 = pick3(st.v[0], e0);
#pragma unroll
        for (int a = 0; a < na; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int r = D == 3 ? a * 3 + b : b;
                fs[r] = ws[r] = INT64_MAX;   // a stencil row outside the grid holds nothing
                if (!(pick3(st.ok[2], a) && pick3(st.ok[1], b))) continue;
                const int64_t c0 = ((int64_t)pick3(st.v[2], a) * g.nc[1] + pick3(st.v[1], b)) * g.nc[0] + x0;
                fs[r] = (int64_t)S.fstart[c0];
                ws[r] = nf + (int64_t)S.wstart[c0];
            }
        const int cnt = S.cnt[i];
        for (int c0 = 1; c0 < cnt; c0 += 8) {
            uint32_t w[3] = {0u, 0u, 0u};
            // the word's eight list entries loaded before any is coded (slots
            // past the count are clamped into the storage and not coded)
            int64_t jw[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const int k = c0 + f < P.cap ? c0 + f : P.cap - 1;
                jw[f] = S.nbr[(int64_t)k * nf + i];
            }
            for (int f = 0; f < 8 && c0 + f < cnt; ++f) {
                const int64_t j = jw[f];
                const bool wl = j >= nf;
                int r = 0;
#pragma unroll
                for (int k = 1; k < NR; ++k)
                    if ((wl ? ws[k] : fs[k]) <= j) r = k;
                const int q = wl ? NR + r : r;
                put12(w, f, (uint32_t)(sp[q] + (int32_t)(j - sb[q])));
            }
            S.pk12[(int64_t)((c0 - 1) >> 3) * nf + i] = make_uint3(w[0], w[1], w[2]);
        }
    }
};

// Wall rows: fluid particles only, no self.
template <int D>
struct BuildWall {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int which) {
        ROW;
        const int64_t w = i;
        if (w >= P.nw) return;
        const Grid &g = P.grid;
        const int64_t iw = P.nf + w, nw = P.nw;
        const Pos x = mkpos(which == POS_XS ? S.xs : S.x);
        const int32_t *items = nullptr;   // the fluid is in the cell order of these positions
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
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    if (!(st.ok[2][a] && st.ok[1][b] && st.ok[0][e])) continue;
                    const int64_t cell = stencil_cell(g, st, a, b, e);
                    // kScanBatch candidates at a time: their positions are
                    // loaded before any is tested (a dependent round trip
                    // per candidate made the walls next to the fluid a
                    // chain of ~475 of them); the set and its order are
                    // those of one candidate at a time
                    const uint32_t t1 = S.fstart[cell + 1];
                    for (uint32_t t = S.fstart[cell]; t < t1; t += kScanBatch) {
                        double xj[kScanBatch][3];
#pragma unroll
                        for (int u = 0; u < kScanBatch; ++u) {
                            const uint32_t tu = t + u < t1 ? t + u : t;
                            const int64_t j = items ? (int64_t)items[tu] : (int64_t)tu;
                            for (int k = 0; k < 3; ++k) xj[u][k] = k < D ? x.c[k][j] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < kScanBatch; ++u) {
                            if (t + u >= t1) break;
                            const int64_t j = items ? (int64_t)items[t + u] : (int64_t)(t + u);
                            double d[3] = {0, 0, 0};
                            for (int k = 0; k < D; ++k) d[k] = min_image(xi[k] - xj[u][k], g, k);
                            if (exact_r2<D>(d) < P.R2) {
                                if (c < cap) S.wnbr[(int64_t)c * nw + w] = (int32_t)j;
                                ++c;
                            }
                        }
                    }
                }
        if (c > cap) {
            atomicOr(&S.ctl->overflow, 1);
            atomicMax(&S.ctl->maxcnt, c);
        }
        S.wcnt[w] = c < cap ? c : cap;
    }
};

// ------------------------------------------------------------ wall normals
// Section 3.4.1: n*_w = -sum_j (m_j/rho0) grad_w W_wj over wall neighbours,
// zeroed below 1/(4h), else made unit; then n_w = sum_j (m_j/rho0) n*_j W_wj,
// made unit (a length below 1e-9 is the rounding residue of opposite layers
// cancelling and is set to zero).  Once per case, from the wall cells.
template <int KER, int D>
struct WallNormals {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int pass) {
        ROW;
        const int64_t w = i;
        if (w >= P.nw) return;
        const Grid &g = P.grid;
        const int64_t nf = P.nf, iw = nf + w, nw = P.nw;
        Kern<KER, D, double> K(P.h);
        const Pos x = mkpos(S.x);
        double *ns[3] = {S.tmp, S.tmp + nw, S.tmp + 2 * nw};
        double xi[3] = {0, 0, 0};
        int ci[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) {
            xi[k] = x.c[k][iw];
            ci[k] = cell_coord(xi[k], g, k);
        }
        Stencil st;
        make_stencil<D>(g, ci, st);
        double a[3] = {0, 0, 0};
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    if (!(st.ok[2][aa] && st.ok[1][b] && st.ok[0][e])) continue;
                    const int64_t cell = stencil_cell(g, st, aa, b, e);
                    for (uint32_t t = S.wstart[cell]; t < S.wstart[cell + 1]; ++t) {
                        const int64_t j = nf + t;
                        double d[3] = {0, 0, 0};
                        for (int k = 0; k < D; ++k) d[k] = min_image(xi[k] - x.c[k][j], g, k);
                        const double r2 = exact_r2<D>(d);
                        if (!(r2 < P.R2)) continue;
                        const double r = sqrt(r2), V = S.m[j] / P.rho0;
                        if (pass == 0) {
                            const double f = K.dwr(r);
                            for (int k = 0; k < D; ++k) a[k] -= V * f * d[k];
                        } else {
                            const double W = K.w(r);
                            for (int k = 0; k < D; ++k) a[k] += V * ns[k][t] * W;
                        }
                    }
                }
        double mag2 = 0.0;
        for (int k = 0; k < D; ++k) mag2 += a[k] * a[k];
        const double mag = sqrt(mag2);
        for (int k = 0; k < D; ++k) {
            if (pass == 0) ns[k][w] = mag < 1.0 / (4.0 * P.h) ? 0.0 : a[k] / mag;
            else S.nrm[k][w] = mag > 1e-9 ? a[k] / mag : 0.0;
        }
    }
};


// ---------------------------------------------------------- wall velocity
// eq. vf: Shepard average of the fluid velocity with a kernel of smoothing
// length h/2; eq. vg-adami: no-slip ghost 2 u_wall - avg (at r^n, from u),
// and at r* (from u*) the slip form avg unless the case asks for the
// no-slip form there too; eq. vg-no-normal: any part into the solid is
// removed.
template <int KER, int D, typename R>
struct WallVelocity {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int which) {
        const int slip = which == POS_XS && !P.ustar_noslip;
        ROW;
        const int64_t w = i;
        if (w >= P.nw) return;
        const int64_t iw = P.nf + w;
        Kern<KER, D, R> K(0.5 * P.h);
        const Pos x = mkpos(which == POS_XS ? S.xs : S.x);
        double *const *uf = which == POS_XS ? S.us : S.u;
        double xi[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) xi[k] = x.c[k][iw];
        R num[3] = {0, 0, 0}, den = R(0);
        const int c = S.wcnt[w];
        // The kernel has smoothing length h/2: a fluid neighbour past its
        // support has W = 0 exactly and adds exact zeros (the sums start at
        // +0), so its velocity is not gathered; the sums are the same bits.
        for (int k0 = 0; k0 < c; k0 += kPairBatch) {
            int64_t fb[kPairBatch];
            double xj[kPairBatch][3], ub[kPairBatch][3];
            batch_slots(S.wnbr, P.nw, w, k0, c, P.cap, iw, fb);
            batch_pos<D>(x, fb, xj);
            R Wb[kPairBatch];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                R d[3], r2;
                pair_diff_v<D, R>(P.grid, xi, xj[t], d, r2);
                Wb[t] = k0 + t < c ? K.w(sqrt(r2)) : R(0);
            }
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t)
                for (int a = 0; a < D; ++a) ub[t][a] = Wb[t] != R(0) ? uf[a][fb[t]] : 0.0;
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                if (k0 + t >= c) break;
                const R W = Wb[t];
                for (int a = 0; a < D; ++a) num[a] += (R)ub[t][a] * W;
                den += W;
            }
        }
        double v[3] = {0, 0, 0}, vn = 0.0;
        if (plain32(P)) {
            float vf[3] = {0.f, 0.f, 0.f}, vnf = 0.f;
            for (int a = 0; a < D; ++a) {
                const float avg = den > R(0) ? (float)num[a] / (float)den : 0.f;
                vf[a] = slip ? avg : 2.f * (float)S.wallu[a][w] - avg;
                vnf += vf[a] * (float)S.nrm[a][w];
            }
            if (vnf < 0.f)
                for (int a = 0; a < D; ++a) vf[a] -= vnf * (float)S.nrm[a][w];
            for (int a = 0; a < D; ++a) uf[a][iw] = vf[a];
            return;
        }
        for (int a = 0; a < D; ++a) {
            const double avg = den > R(0) ? (double)num[a] / (double)den : 0.0;
            v[a] = slip ? avg : 2.0 * S.wallu[a][w] - avg;
            vn += v[a] * S.nrm[a][w];
        }
        if (vn < 0.0)
            for (int a = 0; a < D; ++a) v[a] -= vn * S.nrm[a][w];
        for (int a = 0; a < D; ++a) uf[a][iw] = v[a];
    }
};

// --------------------------------------------------------------- predictor
// Viscous (eq. mom:sph:visc), artificial viscosity (eq. mom:sph:av, read as
// Monaghan's Pi_ij = -alpha h c_ref mu_ij / rho_bar for u_ij.r_ij < 0,
// force -sum m_j Pi_ij gradW), artificial stress (eq. mom:sph:gtvf:stress:
// sum m_j (A_i/rho_i^2 + A_j/rho_j^2).gradW, A = rho u (x) (u~ - u), A = 0 on
// walls) and gravity; then r* = r^n + dt u~^n (eq. int:rnp1, wrapped) and
// u* = u^n + dt f (eq. int:vint).
template <int KER, int D, typename R>
struct Predictor {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.nf) return;
        Kern<KER, D, R> K(P.h);
        const int64_t nf = P.nf;
        const Pos x = mkpos(S.x), u = mkpos(S.u), ut = mkpos(S.ut);
        double xi[3] = {0, 0, 0}, ui_d[3] = {0, 0, 0};
        R ui[3] = {0, 0, 0}, si[3] = {0, 0, 0};
        const R rhoi = (R)S.rho[i];
        for (int k = 0; k < D; ++k) {
            xi[k] = x.c[k][i];
            ui_d[k] = u.c[k][i];
            ui[k] = (R)ui_d[k];
            si[k] = (R)(ut.c[k][i] - u.c[k][i]);   // u~ - u
        }
        // A_i / rho_i^2 = (u_i / rho_i) (x) (u~_i - u_i)
        const R inv_rhoi = R(1) / rhoi;
        const R eps = (R)P.eps_h, nu4 = (R)(4.0 * P.nu), avc = (R)(P.alpha * P.h * P.c_ref);
        R fv[3] = {0, 0, 0}, fa[3] = {0, 0, 0}, fsr[3] = {0, 0, 0};
        const int c = S.cnt[i];
        // the pair loop over one record layout (the 64-byte FP32-sum record
        // when every particle has the same mass)
        auto pairs = [&](auto tag) {
            using Rec = decltype(tag);
            constexpr bool no_mass = std::is_same<Rec, PredRecS>::value;
            const Rec *prec = (const Rec *)S.prec;
            for (int k0 = 1; k0 < c; k0 += kPairBatch) {
                int64_t jb[kPairBatch];
                double xj[kPairBatch][3], ub[kPairBatch][3];
                R sb[kPairBatch][3], mb[kPairBatch], rhob[kPairBatch];
                batch_slots(S.nbr, nf, i, k0, c, P.cap, i, jb);
                // one record per neighbour: positions, velocities in FP64 in
                // every mode (their pair differences are small against the
                // velocities and are formed before any rounding to the working
                // precision), u~ (0 for walls, whose term is not formed), and
                // mass and density in the working precision
                Rec rb[kPairBatch];
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) rb[t] = prec[jb[t]];
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) {
                    for (int a = 0; a < 3; ++a) {
                        xj[t][a] = rb[t].x[a];
                        ub[t][a] = rb[t].u[a];
                        if constexpr (no_mass) sb[t][a] = rb[t].s[a];
                        else sb[t][a] = (R)(rb[t].ut[a] - rb[t].u[a]);   // u~ - u
                    }
                    if constexpr (no_mass) mb[t] = (R)P.m_uni_f;
                    else mb[t] = rb[t].m;
                    rhob[t] = rb[t].rho;
                }
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) {
                    if (k0 + t >= c) break;
                    const int64_t j = jb[t];
                    R d[3], r2;
                    pair_diff_v<D, R>(P.grid, xi, xj[t], d, r2);
                    const R r = sqrt(r2);
                    const R dw = K.dwr(r);
                    R gw[3];
                    for (int a = 0; a < 3; ++a) gw[a] = dw * d[a];
                    const R F = dw * r2;
                    const R mj = mb[t], rhoj = rhob[t];
                    R uj[3] = {0, 0, 0};
                    for (int a = 0; a < D; ++a) uj[a] = (R)ub[t][a];
                    R uij[3] = {0, 0, 0};
                    for (int a = 0; a < D; ++a) uij[a] = (R)(ui_d[a] - ub[t][a]);
                    const R inv_den = R(1) / (r2 + eps);
                    const R cv = mj * nu4 / (rhoi + rhoj) * F * inv_den;
                    for (int a = 0; a < D; ++a) fv[a] += cv * uij[a];
                    R vr = R(0);
                    for (int a = 0; a < D; ++a) vr += uij[a] * d[a];
                    if (vr < R(0)) {
                        const R mu = vr * inv_den;
                        const R Pi = -avc * mu / (R(0.5) * (rhoi + rhoj));
                        for (int a = 0; a < D; ++a) fa[a] -= mj * Pi * gw[a];
                    }
                    // artificial stress: sum_b (A_i/rho_i^2 + A_j/rho_j^2)_ab gw_b
                    R sgi = R(0);
                    for (int b = 0; b < D; ++b) sgi += si[b] * gw[b];
                    R sgj = R(0), uj_over[3] = {0, 0, 0};
                    if (j < nf) {
                        const R inv_rhoj = R(1) / rhoj;
                        for (int b = 0; b < D; ++b) {
                            sgj += sb[t][b] * gw[b];
                            uj_over[b] = uj[b] * inv_rhoj;
                        }
                    }
                    for (int a = 0; a < D; ++a) fsr[a] += mj * (ui[a] * inv_rhoi * sgi + uj_over[a] * sgj);
                }
            }
        };
        if constexpr (sizeof(R) == 4) {
            if (P.m_uni) pairs(PredRecS{});
            else pairs(PredRecF{});
        } else {
            pairs(PredRecD{});
        }
        const double dt = S.ctl->dt;
        for (int a = 0; a < D; ++a) {
            double f, xn, usn;
            if (plain32(P)) {
                const float dtf = (float)dt, ff = (float)(fv[a] + fa[a] + fsr[a]) + (float)P.g[a];
                f = ff;
                xn = (float)xi[a] + dtf * (float)ut.c[a][i];
                usn = (float)u.c[a][i] + dtf * ff;
            } else {
#pragma clang fp contract(off)
                f = (double)(fv[a] + fa[a] + fsr[a]) + P.g[a];
                xn = xi[a] + dt * ut.c[a][i];
                usn = u.c[a][i] + dt * f;
            }
            S.xs[a][i] = rp(P, wrap_periodic(xn, P.grid, a));
            S.us[a][i] = usn;
            if (P.adaptive_dt) S.vk[a][i] = f;   // completed by the pressure force
        }
    }
};

// Wall-weight word of the mixed mode: fluid index and FP32 weight in one
// 8-byte word, slot-major [cap][nw] like the wall lists.
struct PairF {
    int32_t j;
    float c;
};
// The PPE coefficient cache, group-major: neighbour list slot k >= 1 of row
// i sits at position p = k - 1, in group g = p / 4, lane q = p % 4, at
// element (g * N_f + i) * 4 + q, so one 16-byte (FP32) or 32-byte (FP64)
// load brings four consecutive coefficients of a row and a wavefront's 64
// rows read one contiguous block.  The indices sit beside them in the same
// layout: 32-bit, or, for the mixed mode without walls, 16-bit offsets
// j - i modulo N_f when every offset of the step fits (rows are in cell
// order, so neighbours lie within about two cell rows; a periodic wrap is a
// small offset modulo N_f); otherwise the sweep reads the lists.
template <typename R>
struct CoefSlot {
    using T = R;
};
template <typename R>
struct Vec4;
template <>
struct Vec4<float> {
    using T = float4;
};
template <>
struct Vec4<double> {
    using T = double4;
};
struct __align__(8) Off4 {
    int16_t o[4];
};

__device__ __forceinline__ int64_t group_at(int64_t g, int64_t nf, int64_t i) { return g * nf + i; }

__device__ __forceinline__ int32_t offset_index(int64_t i, int16_t o, int64_t nf) {
    int64_t j = i + (int64_t)o;
    if (j < 0) j += nf;
    else if (j >= nf) j -= nf;
    return (int32_t)j;
}

// FP32 copies of the mass and density the mixed-mode pair loops gather
// (they convert each gathered value to FP32 anyway), after the density;
// and the predictor's gather records.  Velocities are gathered in FP64: the
// loops form their pair differences first.
template <typename R>
struct Shadow {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.ntot) return;
        if (sizeof(R) == 4 && P.m_uni) {
            PredRecS rec;
            for (int a = 0; a < 3; ++a) {
                const bool on = a < P.dim;
                rec.x[a] = on ? S.x[a][i] : 0.0;
                rec.u[a] = on ? S.u[a][i] : 0.0;
                rec.s[a] = on && i < P.nf ? (float)(S.ut[a][i] - S.u[a][i]) : 0.0f;
            }
            rec.rho = (float)S.rho[i];
            ((PredRecS *)S.prec)[i] = rec;
        } else {
            using Rec = typename std::conditional<sizeof(R) == 4, PredRecF, PredRecD>::type;
            Rec rec;
            for (int a = 0; a < 3; ++a) {
                const bool on = a < P.dim;
                rec.x[a] = on ? S.x[a][i] : 0.0;
                rec.u[a] = on ? S.u[a][i] : 0.0;
                rec.ut[a] = on && i < P.nf ? S.ut[a][i] : 0.0;
            }
            rec.m = (R)S.m[i];
            rec.rho = (R)S.rho[i];
            ((Rec *)S.prec)[i] = rec;
        }
        if constexpr (sizeof(R) == 4) {
            S.m32[i] = (float)S.m[i];
            S.rho32[i] = (float)S.rho[i];
        }
    }
};

template <typename R>
struct CoefSeed {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.ntot) return;
        using Rec = typename std::conditional<sizeof(R) == 4, CoefRecF, CoefRecD>::type;
        Rec rec;
        for (int a = 0; a < 3; ++a) {
            const bool on = a < P.dim;
            rec.x[a] = on ? S.xs[a][i] : 0.0;
            rec.u[a] = on ? S.us[a][i] : 0.0;
        }
        rec.m = (R)S.m[i];
        rec.rho = (R)S.rho[i];
        ((Rec *)S.prec)[i] = rec;
    }
};

template <typename R>
struct CorrSeed {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.ntot) return;
        if (sizeof(R) == 4 && P.pgrad == SISPH_SYMM) {
            CorrRecS rec;
            for (int a = 0; a < 3; ++a) rec.x[a] = a < P.dim ? S.xs[a][i] : 0.0;
            const double rho = S.rho[i];
            rec.q = (float)(S.p[0][i] / (rho * rho));
            rec.m = (float)S.m[i];
            ((CorrRecS *)S.prec)[i] = rec;
            return;
        }
        CorrRec rec;
        for (int a = 0; a < 3; ++a) rec.x[a] = a < P.dim ? S.xs[a][i] : 0.0;
        rec.p = S.p[0][i];
        rec.rho = S.rho[i];
        rec.m = (double)(R)S.m[i];
        ((CorrRec *)S.prec)[i] = rec;
    }
};

// ------------------------------------------------- PPE RHS and coefficients
// eq. sph-ppe / coeff / coeff1 at r*: RHS_i = sum -m_j/(rho_j dt) u*_ij.gradW,
// c_ij = 4 m_j / (rho_i (rho_i + rho_j)) (r_ij.gradW) / (r^2 + eta h^2),
// D_ii = sum_j c_ij (r^2 + eta h^2, not "+ eta^2").  c_ij is stored in list
// order for the sweeps (and the 16-bit offsets where they apply);
// Lambda = max |RHS/D| over non-free-surface rows (wave max, then one
// atomic per wavefront).
template <int KER, int D, typename R>
struct RhsCoef {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int) {
        ROW;
        const int64_t nf = P.nf;
        unsigned long long lam = 0ull;
        double ya = 0.0, yd = 0.0;
        bool wide = false;
        if (i < nf) {
            Kern<KER, D, R> K(P.h);
            const Pos xs = mkpos(S.xs), us = mkpos(S.us);
            double xi[3] = {0, 0, 0}, usi[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) {
                xi[k] = xs.c[k][i];
                usi[k] = us.c[k][i];
            }
            const R rhoi = (R)S.rho[i], eps = (R)P.eps_h, inv_dt = (R)(1.0 / S.ctl->dt);
            R s = R(0), Dg = R(0);
            const int c = S.cnt[i];
            // a batch of kPairBatch = 4 slots is one group of coefficients
            // (and indices or offsets), written with one store each
            static_assert(kPairBatch == 4, "one coefficient group per batch");
            using Rec = typename std::conditional<sizeof(R) == 4, CoefRecF, CoefRecD>::type;
            const Rec *crec = (const Rec *)S.prec;
            for (int k0 = 1; k0 < c; k0 += kPairBatch) {
                int64_t jb[kPairBatch];
                double xj[kPairBatch][3], usb[kPairBatch][3];
                R mb[kPairBatch], rhob[kPairBatch];
                batch_slots(S.nbr, nf, i, k0, c, P.cap, i, jb);
                // one record per neighbour; u* in FP64: u*_ij is formed
                // before rounding (the RHS is the divergence of a nearly
                // solenoidal field, a sum of terms that mostly cancel)
                Rec rb[kPairBatch];
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) rb[t] = crec[jb[t]];
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) {
                    for (int a = 0; a < 3; ++a) {
                        xj[t][a] = rb[t].x[a];
                        usb[t][a] = rb[t].u[a];
                    }
                    mb[t] = rb[t].m;
                    rhob[t] = rb[t].rho;
                }
                R c4[4] = {R(0), R(0), R(0), R(0)};
                int32_t j4[4] = {(int32_t)i, (int32_t)i, (int32_t)i, (int32_t)i};
                int16_t o4[4] = {0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) {
                    if (k0 + t >= c) break;
                    const int64_t j = jb[t];
                    R d[3], r2;
                    pair_diff_v<D, R>(P.grid, xi, xj[t], d, r2);
                    const R dw = K.dwr(sqrt(r2));
                    const R mj = mb[t], rhoj = rhob[t];
                    R dot = R(0);
                    for (int a = 0; a < D; ++a) dot += (R)(usi[a] - usb[t][a]) * d[a];
                    s -= mj / rhoj * inv_dt * dw * dot;
                    const R cij = R(4) * mj / (rhoi * (rhoi + rhoj)) * (dw * r2) / (r2 + eps);
                    int16_t oq = 0;
                    if (P.compact) {
                        int64_t o = j - i;
                        if (o > nf / 2) o -= nf;
                        else if (o < -(nf / 2)) o += nf;
                        if (o >= -32767 && o <= 32767) oq = (int16_t)o;
                        else wide = true;
                    }
                    c4[t] = cij;
                    j4[t] = (int32_t)j;
                    o4[t] = oq;
                    Dg += cij;
                }
                const int64_t at = group_at((k0 - 1) >> 2, nf, i);
                typename Vec4<R>::T cv;
                cv.x = c4[0];
                cv.y = c4[1];
                cv.z = c4[2];
                cv.w = c4[3];
                ((typename Vec4<R>::T *)S.coef)[at] = cv;
                if (P.compact) {
                    Off4 ov;
                    for (int t = 0; t < 4; ++t) ov.o[t] = o4[t];
                    ((Off4 *)S.cidx)[at] = ov;
                } else {
                    ((int4 *)S.cidx)[at] = make_int4(j4[0], j4[1], j4[2], j4[3]);
                }
            }
            const double rr = (double)s, dd = (double)Dg;
            S.rhs[i] = rr;
            S.dii[i] = dd;
            if (P.packed && sizeof(R) == 4) {
                S.rd32[i] = make_float2((float)rr, (float)dd);   // FP32 sums: exact
                S.cf[i] = c | (S.fs[i] ? (int32_t)0x80000000 : 0);
            }
            if (dd != 0.0 && !S.fs[i])
                lam = (unsigned long long)__double_as_longlong(plain32(P) ? (double)fabsf((float)rr / (float)dd)
                                                                          : fabs(rr / dd));
            if (P.null_space) {
                const double y = S.m[i] * S.rho[i];
                ya = y * rr;
                yd = y * dd;
            }
        }
        if (__any(wide) && (threadIdx.x & 63) == 0) atomicOr(&S.ctl->wide, 1);
        if (P.null_space) {
            // y . RHS and y . D of this workgroup's rows (fixed order), for
            // ProjectFinish; Lambda waits for the projected RHS (ProjectRhs)
            block_sum2(ya, yd);
            if (threadIdx.x == 0) {
                double *pa = S.partial + 2 * nblk;   // the slots of odd sweeps, free until sweep 1
                pa[blk] = ya;
                pa[nblk + blk] = yd;
            }
            return;
        }
        lam = wave_max_u64(lam);   // non-negative doubles order like their bits
        if ((threadIdx.x & 63) == 0 && lam) max_if_larger(&S.ctl->lambda_bits, lam);
    }
};

// Fully periodic cases (SISPH_NULL_PROJECT): constants solve the homogeneous
// PPE and y_i = m_i rho_i is a left null vector of the operator (m_i rho_i
// c_ij is symmetric), so the system is consistent only if y . RHS = 0.  The
// component of the RHS that breaks this is removed once per solve:
// beta = (y . RHS) / (y . D), RHS_i -= beta D_ii; the sweeps of eq. p-sor
// then differ from the unprojected ones by the constant k omega beta only.
// One workgroup per case sums the per-workgroup sums of RhsCoef in a fixed
// order.
struct ProjectFinish {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t, int64_t, int) {
        if (!P.null_space) return;
        const int64_t nb = kind_blocks(P, K_FLUID);
        const double *pa = S.partial + 2 * nb;
        double a = 0.0, b = 0.0;
        for (int64_t k = threadIdx.x; k < nb; k += kBlock) {
            a += pa[k];
            b += pa[nb + k];
        }
        block_sum2(a, b);
        if (threadIdx.x == 0) S.ctl->beta = rp(P, b != 0.0 ? a / b : 0.0);
    }
};

struct ProjectRhs {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        if (!P.null_space) return;
        ROW;
        unsigned long long lam = 0ull;
        if (i < P.nf) {
            const double dd = S.dii[i];
            if (dd != 0.0) {
                const double rr = plain32(P) ? (double)((float)S.rhs[i] - (float)S.ctl->beta * (float)dd)
                                             : S.rhs[i] - S.ctl->beta * dd;
                S.rhs[i] = rr;
                if (!S.fs[i])
                    lam = (unsigned long long)__double_as_longlong(plain32(P) ? (double)fabsf((float)rr / (float)dd)
                                                                              : fabs(rr / dd));
            }
        }
        lam = wave_max_u64(lam);
        if ((threadIdx.x & 63) == 0 && lam) max_if_larger(&S.ctl->lambda_bits, lam);
    }
};

struct CopyP32 {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i < P.ntot) S.p32[i] = (float)S.p[0][i];
    }
};

// ------------------------------------------------------------- PPE sweep
// eq. p-sor with omega: p_i^{k+1} = w (RHS_i + sum_j c_ij p_j^k) / D_ii
// + (1 - w) p_i^k; p = 0 where D_ii = 0 or on free-surface rows (section 3).
// Double-buffered (Jacobi): launch L reads iterate L from buffer L & 1 and
// writes iterate L+1.  Mixed: FP32 c_ij, indices (or 16-bit offsets) and
// the FP32 copy of iterate L; FP64: indices, FP64 coefficients, iterate L.
//
// Stopping (eq. convergence): launch L decides, from the partial sums of
// sweep L-1, whether the solve stopped after L sweeps; the case's workgroup
// 0 takes and records the decision.  No fence or cross-workgroup
// synchronisation is needed (the kernel boundary makes the partials
// visible).  A launch whose solve stopped at an earlier
// count returns at once: stopped_at < L can only have been written by an
// earlier launch, so every wavefront reads the same answer.
//
// First batch: neighbour positions 0..FIRST-1 (FIRST / 4 groups) loaded
// without waiting for the row's count (every group below cap / 4 is inside
// the storage; positions past the count hold stale values and are
// discarded by the select), so the row loads and these loads form one round
// trip.  Longer rows continue kSweepBatchGroups groups at a time.  The sum runs in slot order whatever
// FIRST is, so FIRST (chosen by the autotuner among kSweepFirsts) and the
// workgroup mapping change the speed only, never the result.
// neighbours in the first round trip (multiples of 4); the persistent solve,
// which holds them in registers for the whole solve, takes at least 16
constexpr int kSweepFirsts[kSweepFirstCount] = {8, 16, 20, 24};
constexpr int kSweepBatchGroups = 2;
constexpr int kPartialRegs = 4;   // partial sums per thread in the first pass (1024 workgroups)

// Groups g0 .. g0+NG-1 of a row: coefficients and indices (or offsets),
// group index clamped into the storage (ngroups = cap / 4).  Positions at
// or past the row's count hold stale values that gather_groups discards.
template <typename R, int NG>
__device__ __forceinline__ void load_groups(int64_t i, int64_t nf, int g0, int gmax, const void *coef,
                                            const void *cidx, bool offs, typename Vec4<R>::T (&cc)[NG],
                                            int4 (&jj)[NG], Off4 (&oo)[NG]) {
#pragma unroll
    for (int t = 0; t < NG; ++t) {
        const int g = g0 + t < gmax ? g0 + t : gmax - 1;
        const int64_t at = group_at(g, nf, i);
        cc[t] = ((const typename Vec4<R>::T *)coef)[at];
        if (offs) oo[t] = ((const Off4 *)cidx)[at];
        else jj[t] = ((const int4 *)cidx)[at];
    }
}

// Offsets to indices; when an offset of the step did not fit, the indices
// of the group's slots come from the lists instead.
template <int NG>
__device__ __forceinline__ void resolve_groups(int64_t i, int64_t nf, int g0, int npos, const int32_t *nbr,
                                               bool wide, const Off4 (&oo)[NG], int4 (&jj)[NG]) {
#pragma unroll
    for (int t = 0; t < NG; ++t) {
        int32_t j4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = (g0 + t) * 4 + q;
            if (wide) {
                j4[q] = p < npos ? nbr[(int64_t)(p + 1) * nf + i] : (int32_t)i;
            } else {
                j4[q] = offset_index(i, oo[t].o[q], nf);
            }
        }
        jj[t] = make_int4(j4[0], j4[1], j4[2], j4[3]);
    }
}

// Packed mode: coefficient groups alone, and the 12-bit code words
// (eight positions each; word index clamped into the storage, positions at
// or past the row's count are discarded later).
template <typename R, int NG>
__device__ __forceinline__ void load_coef(int64_t i, int64_t nf, int g0, int gmax, const void *coef,
                                          typename Vec4<R>::T (&cc)[NG]) {
#pragma unroll
    for (int t = 0; t < NG; ++t) {
        const int g = g0 + t < gmax ? g0 + t : gmax - 1;
        cc[t] = ((const typename Vec4<R>::T *)coef)[group_at(g, nf, i)];
    }
}

template <int NW>
__device__ __forceinline__ void load_codes(int64_t i, int64_t nf, int w0, int wmax, const uint3 *pk,
                                           uint3 (&cw)[NW]) {
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        const int w = w0 + t < wmax ? w0 + t : wmax - 1;
        cw[t] = pk[(int64_t)w * nf + i];
    }
}

__device__ __forceinline__ uint32_t code12(const uint3 &w, int f) {
    const uint64_t lo = ((uint64_t)w.y << 32) | w.x, hi = ((uint64_t)w.z << 32) | w.y;
    const int b = 12 * f;
    return (uint32_t)((b < 32 ? lo >> b : hi >> (b - 32)) & 0xfffu);
}

// Iterate values of positions g0*4 .. (g0+NG)*4-1: from the staged copy sp
// by code, or, for a workgroup that is not staged, through the lists; 0 at
// or past npos.
template <typename R, int NG>
__device__ __forceinline__ void packed_gathers(int64_t i, int64_t nf, int g0, int npos, const uint3 *cw,
                                               const R *sp, const int32_t *nbr, const R *q, R (&pv)[NG][4]) {
    if (sp) {
#pragma unroll
        for (int t = 0; t < NG; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = t * 4 + u;
                const uint32_t code = code12(cw[k >> 3], k & 7);
                pv[t][u] = (g0 + t) * 4 + u < npos ? sp[code] : R(0);
            }
    } else {
        int32_t jv[NG][4];
#pragma unroll
        for (int t = 0; t < NG; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = (g0 + t) * 4 + u;
                jv[t][u] = p < npos ? nbr[(int64_t)(p + 1) * nf + i] : (int32_t)i;
            }
#pragma unroll
        for (int t = 0; t < NG; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) pv[t][u] = (g0 + t) * 4 + u < npos ? q[jv[t][u]] : R(0);
    }
}

template <typename R>
__device__ __forceinline__ R vget(const typename Vec4<R>::T &v, int q) {
    return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}
__device__ __forceinline__ int32_t iget(const int4 &v, int q) {
    return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

// Gathered iterate values of the groups' positions (the row's own value
// for positions at or past npos).
template <typename R>
__device__ __forceinline__ R gather_one(int p, int npos, int32_t j, int64_t i, const double *pc, const float *qc) {
    const int32_t jj = p < npos ? j : (int32_t)i;
    if constexpr (sizeof(R) == 4) return qc[jj];
    else return pc[jj];
}

template <typename R, int NG>
__device__ __forceinline__ void issue_gathers(int64_t i, int g0, int npos, const int4 (&jj)[NG], const double *pc,
                                              const float *qc, R (&pv)[NG][4]) {
#pragma unroll
    for (int t = 0; t < NG; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) pv[t][q] = gather_one<R>((g0 + t) * 4 + q, npos, iget(jj[t], q), i, pc, qc);
}

template <typename R, int NG>
__device__ __forceinline__ R sum_gathers(int g0, int npos, const typename Vec4<R>::T (&cc)[NG],
                                         const R (&pv)[NG][4], R s) {
#pragma unroll
    for (int t = 0; t < NG; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = (g0 + t) * 4 + q;
            s += (p < npos ? vget<R>(cc[t], q) : R(0)) * pv[t][q];
        }
    return s;
}

// sum over positions p < npos of the groups, in position (= slot) order
template <typename R, int NG>
__device__ __forceinline__ R gather_groups(int64_t i, int g0, int npos, const typename Vec4<R>::T (&cc)[NG],
                                           const int4 (&jj)[NG], const double *pc, const float *qc, R s) {
    R pv[NG][4];
#pragma unroll
    for (int t = 0; t < NG; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) pv[t][q] = gather_one<R>((g0 + t) * 4 + q, npos, iget(jj[t], q), i, pc, qc);
#pragma unroll
    for (int t = 0; t < NG; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = (g0 + t) * 4 + q;
            s += (p < npos ? vget<R>(cc[t], q) : R(0)) * pv[t][q];
        }
    return s;
}

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

// The stopping decision of eq. convergence from the partial sums of sweep
// L-1, in FP64 (the FP32 mode: every sum, the ratio and the test in FP32).
__device__ __forceinline__ bool stopped_after(const Params &P, const double *partial, int64_t nblk, int L, const PartialLoad &pl,
                              double lam, bool first, Control *ctl) {
    __shared__ double sh[2][kBlock / 64];
    __shared__ int stop_sh;
    const bool f32 = plain32(P);
    double a = 0.0, b = 0.0;
    float af = 0.f, bf = 0.f;
#pragma unroll
    for (int t = 0; t < kPartialRegs; ++t) {
        if (f32) {
            af += (float)pl.a[t];
            bf += (float)pl.b[t];
        } else {
            a += pl.a[t];
            b += pl.b[t];
        }
    }
    if (nblk > (int64_t)kPartialRegs * kBlock) {   // large grids: the rest, in order
        const double *pa = partial + (int64_t)((L - 1) & 1) * 2 * nblk;
        for (int64_t k = threadIdx.x + (int64_t)kPartialRegs * kBlock; k < nblk; k += kBlock) {
            if (f32) {
                af += (float)pa[k];
                bf += (float)pa[nblk + k];
            } else {
                a += pa[k];
                b += pa[nblk + k];
            }
        }
    }
    if (f32) {
        a = wave_sum_f(af);
        b = wave_sum_f(bf);
    } else {
        a = wave_sum(a);
        b = wave_sum(b);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ratio;
        if (f32) {
            float s0 = 0.f, s1 = 0.f;
            for (int t = 0; t < kBlock / 64; ++t) {
                s0 += (float)sh[0][t];
                s1 += (float)sh[1][t];
            }
            float lamf = (float)lam;
            if (P.conv_norm == SISPH_CONV_MEAN) lamf *= (float)P.nf;
            const float scale = lamf > s1 ? lamf : s1;
            const float rf = scale > 0.f ? s0 / scale : (s0 > 0.f ? INFINITY : 0.f);
            a = s0;
            b = s1;
            ratio = rf;
        } else {
            a = 0.0;
            b = 0.0;
            for (int t = 0; t < kBlock / 64; ++t) {
                a += sh[0][t];
                b += sh[1][t];
            }
            if (P.conv_norm == SISPH_CONV_MEAN) lam *= (double)P.nf;
            const double scale = lam > b ? lam : b;
            ratio = scale > 0.0 ? a / scale : (a > 0.0 ? INFINITY : 0.0);
        }
        const bool bad = !isfinite(a) || !isfinite(b);
        const bool below = f32 ? (float)ratio < (float)P.tol : ratio < P.tol;
        bool stop;
        if (P.forced_iters > 0) stop = L >= P.forced_iters;
        else stop = (L >= P.min_iter && below) || L >= P.max_iter;
        stop = stop || bad;
        stop_sh = stop ? 1 : 0;
        if (first) {
            ctl->num = a;
            ctl->den = b;
            ctl->ratio = ratio;
            if (bad) ctl->nonfinite = 1;
            if (stop) {
                ctl->iter = L;
                ctl->done = 1;
                ctl->stopped_at = L;
            }
        }
    }
    __syncthreads();
    return stop_sh != 0;
}

// The damped Jacobi update of eq. p-sor (FP32 throughout in the FP32 mode)
// and the row's terms of the two residual sums.
template <typename R>
__device__ __forceinline__ double psor(const Params &P, double r, R s, double D, double pold) {
    if (plain32(P)) {
        const float w = (float)P.omega;
        return (double)(w * ((float)r + (float)s) / (float)D + (1.f - w) * (float)pold);
    }
    return P.omega * (r + (double)s) / D + (1.0 - P.omega) * pold;
}

// Partial sums |p^{k+1} - p^k| and |p^{k+1}| of the workgroup's rows, valid
// in thread 0 (FP32 sums in the FP32 mode).
__device__ __forceinline__ void residual_partials(const Params &P, bool live, double v, double pold, double &a,
                                                  double &b) {
    if (plain32(P)) {
        float af = live ? fabsf((float)v - (float)pold) : 0.f, bf = live ? fabsf((float)v) : 0.f;
        block_sum2_f(af, bf);
        a = af;
        b = bf;
        return;
    }
    a = live ? fabs(v - pold) : 0.0;
    b = live ? fabs(v) : 0.0;
    block_sum2(a, b);
}

template <typename R, int FIRST, bool PRECHECK>
struct Sweep {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int L) {
        Control *ctl = S.ctl;
        // PRECHECK: a finished solve is detected before any other load (one
        // extra round trip per sweep, but a launch beyond the stop costs
        // almost nothing).  Otherwise the stop flag travels with the first
        // round trip and is tested before the gathers, and a launch beyond
        // the stop reads its row data in vain.
        const int32_t stopped = __hip_atomic_load(&ctl->stopped_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (PRECHECK) {
            if (stopped < L) return;
        }
        // Only the case's first workgroup reduces the partial sums of sweep
        // L-1, decides and records.  The others write iterate L+1 whatever
        // the decision, which is harmless: when the solve stopped after L
        // sweeps the result is iterate L, in the other buffer, and launch
        // L+1 returns at once.  (Every workgroup deciding costs each one a
        // read of all the partial sums: 17 % slower at 160k particles.)
        // The deciding workgroup issues its partial-sum loads with its row
        // loads and decides between issuing its gathers and using them, so
        // the decision costs it no extra round trip.
        const bool decides = L > 0 && blk == 0;
        PartialLoad pl;
        if (decides) load_partials(S.partial, nblk, L, pl);
        const int64_t nf = P.nf;
        const double *pc = S.p[L & 1];
        double *pn = S.p[(L + 1) & 1];
        const float *qc = S.p32 + (L & 1) * P.ntot;
        float *qn = S.p32 + ((L + 1) & 1) * P.ntot;
        const int gmax = P.cap / 4;
        ROW;
        const bool live = i < nf;
        double D = 0.0, r = 0.0, pold = 0.0, v = 0.0;
        int32_t f = 1, c = 0;
        if (P.packed) {
            // The workgroup's staging record (one round trip), then its copy
            // of the iterate its rows reach; codes index the copy.
            constexpr int kStageVals = kStageBytes / (int)sizeof(R);
            __shared__ int32_t rec[kStageRec];
            __shared__ __align__(16) R stage[kStageVals];
            const int NQ = P.dim == 3 ? 18 : 6;
            if ((int)threadIdx.x < 2 * NQ + 2) rec[threadIdx.x] = S.stagerec[blk * kStageRec + threadIdx.x];
            __syncthreads();
            const bool staged = rec[0] != 0;
            const R *q;
            if constexpr (sizeof(R) == 4) q = qc;
            else q = pc;
            if (staged) {
                const int32_t *base = rec + 1, *pos = rec + 1 + NQ;
                const int total = pos[NQ];
                for (int e = threadIdx.x; e < total; e += kBlock) {
                    int sg = 0;
                    while (e >= pos[sg + 1]) ++sg;
                    stage[e] = q[(int64_t)base[sg] + (e - pos[sg])];
                }
            }
            __syncthreads();
            const R *sp = staged ? stage : nullptr;
            // first round trip: row values, the first FP coefficients and
            // their code words (FP: FIRST rounded up to whole code words)
            constexpr int FP = (FIRST + 7) / 8 * 8, NGP = FP / 4, NWP = FP / 8;
            const int wmax = (P.cap + 6) / 8;
            typename Vec4<R>::T cc[NGP];
            uint3 cw[NWP];
            if (live) {
                load_coef<R, NGP>(i, nf, 0, gmax, S.coef, cc);
                if (staged) load_codes<NWP>(i, nf, 0, wmax, S.pk12, cw);
                if constexpr (sizeof(R) == 4) {   // 12 bytes of row words instead of 24
                    const float2 rd = S.rd32[i];
                    const int32_t w = S.cf[i];
                    r = rd.x;
                    D = rd.y;
                    c = w & 0x7fffffff;
                    f = w < 0;
                } else {
                    D = S.dii[i];
                    r = S.rhs[i];
                    f = S.fs[i];
                    c = S.cnt[i];
                }
                pold = pc[i];
            }
            if (stopped < L) return;   // only earlier launches write values below L
            const int npos = c - 1;
            R pv[NGP][4];
            if (live) packed_gathers<R, NGP>(i, nf, 0, npos, cw, sp, S.nbr, q, pv);
            if (decides) {
                const double lam = __longlong_as_double((long long)ctl->lambda_bits);
                if (stopped_after(P, S.partial, nblk, L, pl, lam, true, ctl)) return;
            }
            if (live) {
                R s = sum_gathers<R, NGP>(0, npos, cc, pv, R(0));
                for (int g0 = NGP; 4 * g0 < npos; g0 += 2) {
                    typename Vec4<R>::T cb[2];
                    uint3 cn[1];
                    load_coef<R, 2>(i, nf, g0, gmax, S.coef, cb);
                    if (staged) load_codes<1>(i, nf, g0 / 2, wmax, S.pk12, cn);
                    R pb[2][4];
                    packed_gathers<R, 2>(i, nf, g0, npos, cn, sp, S.nbr, q, pb);
                    s = sum_gathers<R, 2>(g0, npos, cb, pb, s);
                }
                if (D != 0.0 && !f) v = psor<R>(P, r, s, D, pold);
            }
        } else {
            const bool offs = P.compact != 0;
            // set by this step's coefficients: some offset did not fit
            const bool wide = P.compact && ctl->wide;
            // one round trip: row values and the first FIRST / 4 coefficient
            // and index groups
            constexpr int NG = FIRST / 4;
            typename Vec4<R>::T cc[NG];
            int4 jj[NG];
            Off4 oo[NG];
            if (live) {
                load_groups<R, NG>(i, nf, 0, gmax, S.coef, S.cidx, offs, cc, jj, oo);
                D = S.dii[i];
                r = S.rhs[i];
                f = S.fs[i];
                c = S.cnt[i];
                pold = pc[i];
            }
            if (stopped < L) return;   // only earlier launches write values below L
            const int npos = c - 1;    // neighbours besides the row itself
            R pv[NG][4];
            if (live) {
                if (offs) resolve_groups<NG>(i, nf, 0, npos, S.nbr, wide, oo, jj);
                issue_gathers<R, NG>(i, 0, npos, jj, pc, qc, pv);
            }
            // (a solve that stopped earlier returned above: its partials are stale)
            if (decides) {
                const double lam = __longlong_as_double((long long)ctl->lambda_bits);   // fixed during the solve
                if (stopped_after(P, S.partial, nblk, L, pl, lam, true, ctl)) return;
            }
            if (live) {
                R s = sum_gathers<R, NG>(0, npos, cc, pv, R(0));
                for (int g0 = NG; 4 * g0 < npos; g0 += kSweepBatchGroups) {
                    typename Vec4<R>::T cb[kSweepBatchGroups];
                    int4 jb[kSweepBatchGroups];
                    Off4 ob[kSweepBatchGroups];
                    load_groups<R, kSweepBatchGroups>(i, nf, g0, gmax, S.coef, S.cidx, offs, cb, jb, ob);
                    if (offs) resolve_groups<kSweepBatchGroups>(i, nf, g0, npos, S.nbr, wide, ob, jb);
                    s = gather_groups<R, kSweepBatchGroups>(i, g0, npos, cb, jb, pc, qc, s);
                }
                if (D != 0.0 && !f) v = psor<R>(P, r, s, D, pold);
            }
        }
        double a = 0.0, b = 0.0;
        if (live) {
            pn[i] = v;
            if constexpr (sizeof(R) == 4) qn[i] = (float)v;
        }
        residual_partials(P, live, v, pold, a, b);
        if (threadIdx.x == 0) {
            double *pw = S.partial + (int64_t)(L & 1) * 2 * nblk;
            pw[blk] = a;
            pw[nblk + blk] = b;
            if (blk == 0) ctl->iter = L + 1;
        }
    }
};

// ------------------------------------------------- persistent Jacobi solve
// The whole solve of one case without walls in one cooperative launch (all
// workgroups resident, one per 256 rows): each workgroup keeps its rows'
// first FIRST coefficients and neighbour indices, D_ii, RHS, flag, count
// and own iterate in registers for every sweep.  After sweep L every
// workgroup posts L+1 in its own arrival word once its stores have
// completed; workgroup 0 waits for all of them and posts 2 (L+1) + stop in
// one word per XCD, which the others wait for.  Workgroup 0 takes the
// per-launch sweep's decision (before sweep L, whether the solve stopped
// after L sweeps, from sweep L-1's partial sums) while the others run
// sweep L, so the stop is posted after sweep L, as the per-launch path
// returns from launch L+1: sums, their order, the decision and the sweep
// count are bitwise the same.  What other workgroups read during the launch
// (the gathered iterate, the partial sums, these words) is written and read
// with device-scope accesses, which are coherent across XCDs without a
// cache write-back.  A wait that does not end within P.barrier_spins polls
// sets a flag and every workgroup leaves (the host reports the error).
template <typename T>
__device__ __forceinline__ T dev_load(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void dev_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename R, int NG>
__device__ __forceinline__ void gather_dev(int64_t i, int g0, int npos, const int4 (&jj)[NG], const double *pc,
                                           const float *qc, R (&pv)[NG][4]) {
#pragma unroll
    for (int t = 0; t < NG; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = (g0 + t) * 4 + q;
            const int32_t j = p < npos ? iget(jj[t], q) : (int32_t)i;
            if constexpr (sizeof(R) == 4) pv[t][q] = dev_load(qc + j);
            else pv[t][q] = dev_load(pc + j);
        }
}

template <typename R, int FIRST>
__global__ __launch_bounds__(kBlock) void k_ppe_persistent(const Params P, const State S, int limit) {
    Control *ctl = S.ctl;
    const int64_t blk = blockIdx.x, nblk = gridDim.x;
    const int64_t nf = P.nf;
    const bool offs = P.compact != 0;
    const int32_t wide_flag = offs ? ctl->wide : 0;
    const int gmax = P.cap / 4;
    ROW;
    const bool live = i < nf;
    constexpr int NG = FIRST / 4;
    typename Vec4<R>::T cc[NG];
    int4 jj[NG];
    Off4 oo[NG];
    double D = 0.0, r = 0.0, pold = 0.0;
    int32_t f = 1, c = 1;
    if (live) {
        load_groups<R, NG>(i, nf, 0, gmax, S.coef, S.cidx, offs, cc, jj, oo);
        D = S.dii[i];
        r = S.rhs[i];
        f = S.fs[i];
        c = S.cnt[i];
        pold = S.p[0][i];
        if (offs) resolve_groups<NG>(i, nf, 0, c - 1, S.nbr, wide_flag != 0, oo, jj);
    }
    const int npos = c - 1;
    const double lam = __longlong_as_double((long long)ctl->lambda_bits);   // fixed during the solve
    uint32_t *const late_flag = S.sync;
    uint32_t *const arrive = S.sync + kSyncArrive;
    __shared__ int go;
    bool stopped = false;   // workgroup 0, once it recorded the stop
    for (int L = 0; L < limit; ++L) {
        // workgroup 0 decides whether the solve stopped after L sweeps from
        // sweep L-1's partial sums (all posted before the last barrier),
        // while the others already run sweep L; a stop travels with the
        // word posted after sweep L
        if (L > 0 && blk == 0 && !stopped) {
            PartialLoad pl;
            const double *pa = S.partial + (int64_t)((L - 1) & 1) * 2 * nblk;
#pragma unroll
            for (int t = 0; t < kPartialRegs; ++t) {   // nblk <= kPartialRegs * kBlock here
                const int64_t k = threadIdx.x + (int64_t)t * kBlock;
                pl.a[t] = k < nblk ? dev_load(pa + k) : 0.0;
                pl.b[t] = k < nblk ? dev_load(pa + nblk + k) : 0.0;
            }
            stopped = stopped_after(P, S.partial, nblk, L, pl, lam, true, ctl);
        }
        const double *pc = S.p[L & 1];
        double *pn = S.p[(L + 1) & 1];
        const float *qc = S.p32 + (L & 1) * P.ntot;
        float *qn = S.p32 + ((L + 1) & 1) * P.ntot;
        double v = 0.0;
        if (live) {
            R pv[NG][4];
            gather_dev<R, NG>(i, 0, npos, jj, pc, qc, pv);
            R s = sum_gathers<R, NG>(0, npos, cc, pv, R(0));
            for (int g0 = NG; 4 * g0 < npos; g0 += kSweepBatchGroups) {
                typename Vec4<R>::T cb[kSweepBatchGroups];
                int4 jb[kSweepBatchGroups];
                Off4 ob[kSweepBatchGroups];
                load_groups<R, kSweepBatchGroups>(i, nf, g0, gmax, S.coef, S.cidx, offs, cb, jb, ob);
                if (offs) resolve_groups<kSweepBatchGroups>(i, nf, g0, npos, S.nbr, wide_flag != 0, ob, jb);
                R pb[kSweepBatchGroups][4];
                gather_dev<R, kSweepBatchGroups>(i, g0, npos, jb, pc, qc, pb);
                s = sum_gathers<R, kSweepBatchGroups>(g0, npos, cb, pb, s);
            }
            if (D != 0.0 && !f) v = psor<R>(P, r, s, D, pold);
        }
        double a = 0.0, b = 0.0;
        if (live) {
            if constexpr (sizeof(R) == 4) {
                pn[i] = v;
                dev_store(qn + i, (float)v);
            } else {
                dev_store(pn + i, v);
            }
        }
        residual_partials(P, live, v, pold, a, b);
        if (live) pold = v;
        if (threadIdx.x == 0) {
            double *pw = S.partial + (int64_t)(L & 1) * 2 * nblk;
            dev_store(pw + blk, a);
            dev_store(pw + nblk + blk, b);
            if (blk == 0 && !stopped) ctl->iter = L + 1;
        }
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this sweep's stores completed
        __syncthreads();
        if (threadIdx.x == 0) dev_store(arrive + blk, (uint32_t)(L + 1));
        const uint32_t want = 2u * (uint32_t)(L + 1);
        if (blk == 0) {
            bool all = false;
            for (uint32_t spins = 0;; ++spins) {
                bool ok = true;
#pragma unroll
                for (int t = 0; t < kPartialRegs; ++t) {
                    const int64_t k = threadIdx.x + (int64_t)t * kBlock;
                    if (k < nblk && dev_load(arrive + k) < (uint32_t)(L + 1)) ok = false;
                }
                const int give_up = threadIdx.x == 0 && (dev_load(late_flag) != 0u || spins >= P.barrier_spins);
                all = __syncthreads_and(ok);
                const bool quit = __syncthreads_or(give_up);
                if (all || quit) break;
                __builtin_amdgcn_s_sleep(1);
            }
            if (threadIdx.x == 0) {
                if (!all) {
                    dev_store(late_flag, 1u);
                    ctl->barrier_late = 1;
                }
                const bool leave = stopped || !all;
                const uint32_t word = want + (leave ? 1u : 0u);
                for (int x = 0; x < kSyncCopies; ++x) dev_store(S.sync + kSyncBcast + 64 * x, word);
                go = leave ? 0 : 1;
            }
        } else if (threadIdx.x == 0) {
            const uint32_t *w = S.sync + kSyncBcast + 64 * (blk % kSyncCopies);
            uint32_t word = dev_load(w);
            for (uint32_t spins = 0; word < want && dev_load(late_flag) == 0u && spins < P.barrier_spins; ++spins) {
                __builtin_amdgcn_s_sleep(1);
                word = dev_load(w);
            }
            if (word < want) {
                dev_store(late_flag, 1u);
                ctl->barrier_late = 1;
                go = 0;
            } else {
                go = (word & 1u) ? 0 : 1;
            }
        }
        __syncthreads();
        if (!go) break;
    }
}

// The Jacobi solves of several wall-less cases of a batch in one
// cooperative launch: one workgroup per fluid block of every such case (all
// resident), each holding its rows' first FIRST coefficients in registers as
// the single-case persistent solve does.  Every workgroup meets the others
// at one grid barrier per sweep (arrival words, workgroup 0 of the launch
// posting one word per XCD).  Each case keeps its own stopping decision:
// its first workgroup takes it from the case's partial sums exactly as the
// per-launch sweep does, and on a stop posts the case's stop word and counts
// the case as finished; after the barrier the case's workgroups read that
// word and do no further sweep, while still meeting the barriers.  The
// launch ends when every case has stopped (the last barrier's word carries
// the bit), so each case's sums, sweeps and decision are bitwise those it
// would have alone.  On leaving, each case's stop marker is set below every
// sweep count, so per-launch sweeps of the other cases of its batch return
// at once for it.  A wait that does not end within spins polls sets the
// launch's late flag and every workgroup leaves.
constexpr int64_t kBatchStopWords = kBatchSyncStop;   // per-case stop words follow the arrivals
constexpr int kBatchDone = 32;                        // cases stopped so far

template <typename R, int FIRST>
__global__ __launch_bounds__(kBlock) void k_ppe_persistent_batch(const CaseEntry *__restrict__ tab,
                                                                 const int32_t *__restrict__ powner,
                                                                 const int64_t *__restrict__ pfirst, uint32_t *bsync,
                                                                 int ncase, int limit, uint32_t spins) {
    const int64_t gb = blockIdx.x, gn = gridDim.x;
    const int cidx = powner[gb];
    const Params &P = tab[cidx].P;
    const State &S = tab[cidx].S;
    Control *ctl = S.ctl;
    const int64_t blk = gb - pfirst[cidx], nblk = tab[cidx].nblk[K_FLUID];
    const int64_t nf = P.nf;
    const bool offs = P.compact != 0;
    const int32_t wide_flag = offs ? ctl->wide : 0;
    const int gmax = P.cap / 4;
    ROW;
    const bool live = i < nf;
    constexpr int NG = FIRST / 4;
    typename Vec4<R>::T cc[NG];
    int4 jj[NG];
    Off4 oo[NG];
    double D = 0.0, r = 0.0, pold = 0.0;
    int32_t f = 1, c = 1;
    if (live) {
        load_groups<R, NG>(i, nf, 0, gmax, S.coef, S.cidx, offs, cc, jj, oo);
        D = S.dii[i];
        r = S.rhs[i];
        f = S.fs[i];
        c = S.cnt[i];
        pold = S.p[0][i];
        if (offs) resolve_groups<NG>(i, nf, 0, c - 1, S.nbr, wide_flag != 0, oo, jj);
    }
    const int npos = c - 1;
    const double lam = __longlong_as_double((long long)ctl->lambda_bits);   // fixed during the solve
    uint32_t *const late_flag = bsync;
    uint32_t *const arrive = bsync + kSyncArrive;
    uint32_t *const stopw = bsync + kBatchStopWords + cidx;
    __shared__ int go, cdone_sh;
    bool stopped = false;   // the case's first workgroup, once it recorded the stop
    bool cdone = false;     // this workgroup's case has stopped
    for (int L = 0; L < limit; ++L) {
        if (!cdone) {
            if (L > 0 && blk == 0 && !stopped) {
                PartialLoad pl;
                const double *pa = S.partial + (int64_t)((L - 1) & 1) * 2 * nblk;
#pragma unroll
                for (int t = 0; t < kPartialRegs; ++t) {   // nblk <= kPartialRegs * kBlock here
                    const int64_t k = threadIdx.x + (int64_t)t * kBlock;
                    pl.a[t] = k < nblk ? dev_load(pa + k) : 0.0;
                    pl.b[t] = k < nblk ? dev_load(pa + nblk + k) : 0.0;
                }
                stopped = stopped_after(P, S.partial, nblk, L, pl, lam, true, ctl);
                if (stopped && threadIdx.x == 0) {
                    dev_store(stopw, (uint32_t)L);
                    __hip_atomic_fetch_add(bsync + kBatchDone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            const double *pc = S.p[L & 1];
            double *pn = S.p[(L + 1) & 1];
            const float *qc = S.p32 + (L & 1) * P.ntot;
            float *qn = S.p32 + ((L + 1) & 1) * P.ntot;
            double v = 0.0;
            if (live) {
                R pv[NG][4];
                gather_dev<R, NG>(i, 0, npos, jj, pc, qc, pv);
                R s = sum_gathers<R, NG>(0, npos, cc, pv, R(0));
                for (int g0 = NG; 4 * g0 < npos; g0 += kSweepBatchGroups) {
                    typename Vec4<R>::T cb[kSweepBatchGroups];
                    int4 jb[kSweepBatchGroups];
                    Off4 ob[kSweepBatchGroups];
                    load_groups<R, kSweepBatchGroups>(i, nf, g0, gmax, S.coef, S.cidx, offs, cb, jb, ob);
                    if (offs) resolve_groups<kSweepBatchGroups>(i, nf, g0, npos, S.nbr, wide_flag != 0, ob, jb);
                    R pb[kSweepBatchGroups][4];
                    gather_dev<R, kSweepBatchGroups>(i, g0, npos, jb, pc, qc, pb);
                    s = sum_gathers<R, kSweepBatchGroups>(g0, npos, cb, pb, s);
                }
                if (D != 0.0 && !f) v = psor<R>(P, r, s, D, pold);
            }
            double a = 0.0, b = 0.0;
            if (live) {
                if constexpr (sizeof(R) == 4) {
                    pn[i] = v;
                    dev_store(qn + i, (float)v);
                } else {
                    dev_store(pn + i, v);
                }
            }
            residual_partials(P, live, v, pold, a, b);
            if (live) pold = v;
            if (threadIdx.x == 0) {
                double *pw = S.partial + (int64_t)(L & 1) * 2 * nblk;
                dev_store(pw + blk, a);
                dev_store(pw + nblk + blk, b);
                if (blk == 0 && !stopped) ctl->iter = L + 1;
            }
        }
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this sweep's stores completed
        __syncthreads();
        if (threadIdx.x == 0) dev_store(arrive + gb, (uint32_t)(L + 1));
        const uint32_t want = 2u * (uint32_t)(L + 1);
        if (gb == 0) {
            bool all = false;
            for (uint32_t sp = 0;; ++sp) {
                bool ok = true;
#pragma unroll
                for (int t = 0; t < kPartialRegs; ++t) {
                    const int64_t k = threadIdx.x + (int64_t)t * kBlock;
                    if (k < gn && dev_load(arrive + k) < (uint32_t)(L + 1)) ok = false;
                }
                const int give_up = threadIdx.x == 0 && (dev_load(late_flag) != 0u || sp >= spins);
                all = __syncthreads_and(ok);
                const bool quit = __syncthreads_or(give_up);
                if (all || quit) break;
                __builtin_amdgcn_s_sleep(1);
            }
            if (threadIdx.x == 0) {
                if (!all) dev_store(late_flag, 1u);
                const bool leave = !all || dev_load(bsync + kBatchDone) >= (uint32_t)ncase;
                const uint32_t word = want + (leave ? 1u : 0u);
                for (int x = 0; x < kSyncCopies; ++x) dev_store(bsync + kSyncBcast + 64 * x, word);
                go = leave ? 0 : 1;
            }
        } else if (threadIdx.x == 0) {
            const uint32_t *w = bsync + kSyncBcast + 64 * (gb % kSyncCopies);
            uint32_t word = dev_load(w);
            for (uint32_t sp = 0; word < want && dev_load(late_flag) == 0u && sp < spins; ++sp) {
                __builtin_amdgcn_s_sleep(1);
                word = dev_load(w);
            }
            if (word < want) {
                dev_store(late_flag, 1u);
                go = 0;
            } else {
                go = (word & 1u) ? 0 : 1;
            }
        }
        if (threadIdx.x == 0) cdone_sh = dev_load(stopw) != 0xffffffffu;
        __syncthreads();
        cdone = cdone_sh != 0;
        if (!go) break;
    }
    // later per-launch sweeps of the batch return at once for this case
    if (blk == 0 && threadIdx.x == 0 && stopped) ctl->stopped_at = -1;
}

// eq. p-shepard: p_w = [sum_f p_f W_wf + (g - a_w) . sum_f rho_f r_wf W_wf]
// / sum_f W_wf over fluid neighbours (static wall: a_w = 0); 0 without
// neighbours; clamped at 0 on free-surface problems.  Positions and
// densities are fixed during the solve, so once per step (at r*) WallCoef
// caches, in list order, the normalised weights a_wf = W_wf / sum W (with
// the fluid index in the mixed mode, FP32 weight) and the hydrostatic term
// h_w = g . sum rho_f r_wf W_wf / sum W; each sweep then forms
// p_w = sum_f a_wf p_f + h_w.
// In the FP32-sum modes the words go where the per-sweep pass reads them
// with no waste: each wall row with fluid neighbours has its c_w words in
// one run, the runs one after the other in wall order (a slot-major layout
// would fetch every line that any row of its sixteen holds a slot in, about
// three times the words on a walled 3D case).  The workgroup's offsets come
// from WallBlocks; a row's place within its workgroup is an exclusive scan
// over its rows of (has neighbours, c_w).
template <int KER, int D, typename R>
struct WallCoef {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        const int64_t w = i;
        uint32_t off = 0;
        if constexpr (sizeof(R) == 4) {
            __shared__ uint32_t wave_a[kBlock / 64], wave_c[kBlock / 64];
            const uint32_t cw = w < P.nw ? (uint32_t)S.wcnt[w] : 0u, aw = cw > 0u;
            uint32_t ia = aw, ic = cw;   // inclusive scan over the wave
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t ta = __shfl_up(ia, o, 64), tc = __shfl_up(ic, o, 64);
                if (lane >= o) {
                    ia += ta;
                    ic += tc;
                }
            }
            if (lane == 63) {
                wave_a[wave] = ia;
                wave_c[wave] = ic;
            }
            __syncthreads();
            uint32_t ba = S.wsum[2 * blk], bc = S.wsum[2 * blk + 1];
            for (int v = 0; v < wave; ++v) {
                ba += wave_a[v];
                bc += wave_c[v];
            }
            off = bc + ic - cw;
            if (w < P.nw) {
                S.woffw[w] = off;
                if (aw) S.wrow[ba + ia - aw] = make_uint2((uint32_t)w, off);
            }
        }
        if (w >= P.nw) return;
        const int64_t iw = P.nf + w, nw = P.nw;
        Kern<KER, D, R> K(P.h);
        const Pos xs = mkpos(S.xs);
        double xi[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) xi[k] = xs.c[k][iw];
        R sr[3] = {0, 0, 0}, sw = R(0);
        const int c = S.wcnt[w];
        // kPairBatch slots at a time (indices, then positions and
        // densities, then the terms in slot order)
        for (int k0 = 0; k0 < c; k0 += kPairBatch) {
            int64_t fb[kPairBatch];
            double xj[kPairBatch][3], rb[kPairBatch];
            batch_slots(S.wnbr, nw, w, k0, c, P.cap, iw, fb);
            batch_pos<D>(xs, fb, xj);
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) rb[t] = S.rho[fb[t]];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                if (k0 + t >= c) break;
                R d[3], r2;
                pair_diff_v<D, R>(P.grid, xi, xj[t], d, r2);
                const R W = K.w(sqrt(r2));
                const R rw = (R)rb[t] * W;
                for (int a = 0; a < D; ++a) sr[a] += rw * d[a];
                sw += W;
            }
        }
        double h = 0.0;
        const R inv = sw > R(0) ? R(1) / sw : R(0);
        if (sw > R(0)) {
            double gs = 0.0;
            for (int a = 0; a < D; ++a) gs += P.g[a] * (double)sr[a];
            h = gs / (double)sw;
        }
        S.wh[w] = rp(P, h);
        // second pass: the normalised weights (the kernel values again, in
        // the same order, rather than holding them in registers)
        for (int k0 = 0; k0 < c; k0 += kPairBatch) {
            int64_t fb[kPairBatch];
            double xj[kPairBatch][3];
            batch_slots(S.wnbr, nw, w, k0, c, P.cap, iw, fb);
            batch_pos<D>(xs, fb, xj);
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                const int k = k0 + t;
                if (k >= c) break;
                R d[3], r2;
                pair_diff_v<D, R>(P.grid, xi, xj[t], d, r2);
                const R a = K.w(sqrt(r2)) * inv;
                if constexpr (sizeof(R) == 4) ((PairF *)S.wcoef)[(int64_t)off + k] = PairF{(int32_t)fb[t], a};
                else ((double *)S.wcoef)[(int64_t)k * nw + w] = a;
            }
        }
    }
};

// During the solve it writes the wall slots of iterate L (which sweep L
// reads); with final set, the wall slots of p[0] after the final pressure
// has been settled there.
// Cached wall weights and fluid indices of slots k0 .. k0+kPairBatch-1 of
// wall row w (slot clamped into the storage).
// Wall workgroups the sweeps visit.  A wall row without fluid neighbours
// at r* is in no fluid row's list either (the neighbour relation is
// symmetric), so no sweep reads its pressure: the per-sweep wall pass skips
// workgroups made only of such rows (the final pass after the solve still
// covers every wall row).  WallFlags marks each wall workgroup; WallBlocks
// (one workgroup per case) lists the marked ones in order.
// WallFlags also counts the workgroup's rows with neighbours and their
// entries, which WallBlocks turns into exclusive prefixes in place (the
// placement of the FP32 weight runs).
struct WallFlags {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        __shared__ uint32_t wave_a[kBlock / 64], wave_c[kBlock / 64];
        ROW;
        uint32_t c = i < P.nw ? (uint32_t)S.wcnt[i] : 0u, a = c > 0u;
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            wave_a[threadIdx.x >> 6] = a;
            wave_c[threadIdx.x >> 6] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t ta = 0, tc = 0;
            for (int v = 0; v < kBlock / 64; ++v) {
                ta += wave_a[v];
                tc += wave_c[v];
            }
            S.wflag[blk] = ta > 0;
            S.wsum[2 * blk] = ta;
            S.wsum[2 * blk + 1] = tc;
        }
    }
};

struct WallBlocks {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t, int64_t, int) {
        __shared__ int32_t sh[kBlock];
        const int64_t nb = (P.nw + kBlock - 1) / kBlock;
        const int64_t chunk = (nb + kBlock - 1) / kBlock;
        const int64_t b0 = threadIdx.x * chunk, b1 = b0 + chunk < nb ? b0 + chunk : nb;
        int32_t n = 0;
        for (int64_t b = b0; b < b1; ++b) n += S.wflag[b] != 0;
        sh[threadIdx.x] = n;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {   // inclusive scan of the counts
            const int32_t v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += v;
            __syncthreads();
        }
        int32_t pos = sh[threadIdx.x] - n;
        for (int64_t b = b0; b < b1; ++b)
            if (S.wflag[b] != 0) S.wblk[1 + pos++] = (int32_t)b;
        if (threadIdx.x == kBlock - 1) S.wblk[0] = sh[kBlock - 1];
        // exclusive prefixes of the (rows, entries) counts, chunk by chunk
        __shared__ uint32_t sa[kBlock], sc[kBlock];
        uint32_t ta = 0, tc = 0;
        for (int64_t b = b0; b < b1; ++b) {
            ta += S.wsum[2 * b];
            tc += S.wsum[2 * b + 1];
        }
        sa[threadIdx.x] = ta;
        sc[threadIdx.x] = tc;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const uint32_t va = threadIdx.x >= off ? sa[threadIdx.x - off] : 0u;
            const uint32_t vc = threadIdx.x >= off ? sc[threadIdx.x - off] : 0u;
            __syncthreads();
            sa[threadIdx.x] += va;
            sc[threadIdx.x] += vc;
            __syncthreads();
        }
        uint32_t ra = sa[threadIdx.x] - ta, rc = sc[threadIdx.x] - tc;
        for (int64_t b = b0; b < b1; ++b) {
            const uint32_t a = S.wsum[2 * b], c = S.wsum[2 * b + 1];
            S.wsum[2 * b] = ra;
            S.wsum[2 * b + 1] = rc;
            ra += a;
            rc += c;
        }
        if (threadIdx.x == kBlock - 1) {
            S.wsum[2 * nb] = sa[kBlock - 1];
            S.wsum[2 * nb + 1] = sc[kBlock - 1];
            S.wrow[sa[kBlock - 1]] = make_uint2(~0u, sc[kBlock - 1]);
        }
    }
};

// FP64: weights and fluid indices of slots k0 .. k0+kPairBatch-1 of the
// [cap][nw] weights and lists (slot clamped into the storage).
__device__ __forceinline__ void wall_words(const State &S, int64_t nw, int64_t w, int k0, int cap,
                                           double (&cb)[kPairBatch], int32_t (&jr)[kPairBatch]) {
#pragma unroll
    for (int t = 0; t < kPairBatch; ++t) {
        const int k = k0 + t < cap ? k0 + t : cap - 1;
        const int64_t at = (int64_t)k * nw + w;
        cb[t] = ((const double *)S.wcoef)[at];
        jr[t] = S.wnbr[at];
    }
}

// FP32 sums: sum_f a_wf p_f of one wall row over its run of c words at a0,
// kWallLanes lanes per row.  Lane q takes words q, q + kWallLanes, ... (the
// group reads consecutive words), kWallWords of them per batch, and adds
// its terms in word order; the row's sum is the butterfly over the group
// ((s0 + s1) + (s2 + s3)) + ..., the same bits on every lane of the group
// (IEEE addition commutes).  Words past the run are clamped to its last
// one (word 0 of the buffer for an empty run) and add nothing.
constexpr int kWallLanes = 4, kWallWords = 8;

__device__ __forceinline__ float wall_run_sum(const State &S, const float *qc, int64_t a0, int c, int q,
                                              int64_t iw) {
    const PairF *wd = (const PairF *)S.wcoef + a0;
    const int last = c > 0 ? c - 1 : 0;
    float s = 0.0f;
    for (int b0 = 0;; b0 += kWallLanes * kWallWords) {
        float cb[kWallWords], v[kWallWords];
        int32_t jr[kWallWords];
#pragma unroll
        for (int t = 0; t < kWallWords; ++t) {
            const int k = b0 + q + kWallLanes * t;
            const PairF e = wd[k < c ? k : last];
            cb[t] = e.c;
            jr[t] = e.j;
        }
#pragma unroll
        for (int t = 0; t < kWallWords; ++t) {
            const int k = b0 + q + kWallLanes * t;
            v[t] = qc[k < c ? (int64_t)jr[t] : iw];   // iw: a valid index, term not added
        }
#pragma unroll
        for (int t = 0; t < kWallWords; ++t) {
            const int k = b0 + q + kWallLanes * t;
            const float acc = fmaf(cb[t], v[t], s);
            s = k < c ? acc : s;
        }
        if (b0 + kWallLanes * kWallWords >= c) break;   // the same on the row's four lanes
    }
    for (int o = 1; o < kWallLanes; o <<= 1) s += __shfl_xor(s, o);
    return s;
}

template <typename R>
struct WallPressure {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int L,
                                               int final) {
        const int64_t nw = P.nw, nb = (nw + kBlock - 1) / kBlock;
        // FP32 sums: during the solve the rows with fluid neighbours
        // (compact, in the first launch slots); the final pass every wall
        // row.  A workgroup takes kBlock / kWallLanes rows at a time,
        // striding by the grid (nblk workgroups: during the solve at most
        // kWallRunBlocks, enough for the rows near the fluid in one round on
        // the large cases).  The row count and the first row's entry are
        // read with the stop flag rather than after it (wrow has nw + 1
        // entries; one past the rows is read and not used).
        const int64_t stride = nblk * (kBlock / kWallLanes);
        int64_t r = blk * (kBlock / kWallLanes) + threadIdx.x / kWallLanes;
        int64_t listed = 0;
        uint2 e = make_uint2(0u, 0u), e1 = e;
        if (sizeof(R) == 4 && !final) {
            listed = S.wsum[2 * nb];
            const int64_t rc = r < nw ? r : nw;
            e = S.wrow[rc];
            e1 = S.wrow[rc < nw ? rc + 1 : nw];
        }
        if (!final && __hip_atomic_load(&S.ctl->stopped_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < L) return;
        const int par = final ? 0 : (L & 1);
        double *pc = S.p[par];
        float *qc = S.p32 + par * P.ntot;
        if constexpr (sizeof(R) == 4) {
            const int64_t rows = final ? nw : listed;
            const int q = threadIdx.x & (kWallLanes - 1);
            for (; r < rows; r += stride) {
                int64_t w, a0;
                int c;
                if (final) {
                    w = r;
                    c = S.wcnt[w];
                    a0 = c > 0 ? (int64_t)S.woffw[w] : 0;
                } else {
                    w = e.x;
                    a0 = e.y;
                    c = (int)(e1.y - e.y);
                    if (r + stride < rows) {
                        e = S.wrow[r + stride];
                        e1 = S.wrow[r + stride + 1];
                    }
                }
                const double h = S.wh[w];
                const int64_t iw = P.nf + w;
                const float sp = wall_run_sum(S, qc, a0, c, q, iw);
                double pw = plain32(P) ? (double)(sp + (float)h) : (double)sp + h;
                if (P.free_surface && pw < 0.0) pw = 0.0;
                if (q == 0) {
                    pc[iw] = pw;
                    qc[iw] = (float)pw;
                }
            }
            return;
        }
        if (!final) {
            if (blk >= S.wblk[0]) return;   // the listed workgroups take the first launch slots
            blk = S.wblk[1 + blk];
        }
        ROW;
        const int64_t w = i;
        if (w >= nw) return;
        const int64_t iw = P.nf + w;
        const int c = S.wcnt[w];
        // kPairBatch slots at a time: weights and indices, then the gathered
        // iterate values, then the terms in slot order; the first batch's
        // words are loaded with the count, without waiting for it.
        // The first batch runs whatever the count (its gathers read the
        // row's own slot and add nothing when c = 0), and the terms are
        // selected rather than branched over, so no load waits behind a
        // branch.  sp + 0 leaves sp unchanged (sp starts at +0 and never
        // becomes -0), so the sum is the plain slot-order sum.
        double sp = 0.0;
        double cb[kPairBatch];
        int32_t jr[kPairBatch];
        wall_words(S, nw, w, 0, P.cap, cb, jr);
        for (int k0 = 0;;) {
            double q[kPairBatch];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) q[t] = pc[k0 + t < c ? (int64_t)jr[t] : iw];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                const double acc = fma(cb[t], q[t], sp);
                sp = k0 + t < c ? acc : sp;
            }
            k0 += kPairBatch;
            if (k0 >= c) break;
            wall_words(S, nw, w, k0, P.cap, cb, jr);
        }
        double pw = sp + S.wh[w];
        if (P.free_surface && pw < 0.0) pw = 0.0;
        pc[iw] = pw;
        qc[iw] = (float)pw;
    }
};

// After the solve: the final iterate into p[0] (it is in p[iters & 1]).
// In the mixed mode the FP32 copy moves too: the final wall pass reads it.
struct SettlePressure {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i < P.ntot && (S.ctl->iter & 1)) {
            S.p[0][i] = S.p[1][i];
            if (f32_sums(P.precision)) S.p32[i] = S.p32[P.ntot + i];
        }
    }
};

// max p over the fluid, needed only until p_ref is set (first solve)
struct PMax {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        if (S.ctl->p_ref_set) return;
        ROW;
        unsigned long long k = i < P.nf ? order_key(S.p[0][i]) : 0ull;
        k = wave_max_u64(k);
        if ((threadIdx.x & 63) == 0 && k) max_if_larger(&S.ctl->pmax_key, k);
    }
};

// p_ref for internal flows: twice the largest pressure after the first
// solve, then held (section 2.1).
struct PrefFinish {
    static __device__ __forceinline__ void run(const Params &, const State &S, int64_t, int64_t, int) {
        Control *c = S.ctl;
        if (threadIdx.x == 0 && !c->p_ref_set) {
            c->p_ref = 2.0 * order_val(c->pmax_key);   // exact for an FP32 value too
            c->p_ref_set = 1;
        }
    }
};

// ----------------------------------------------- pressure force, correction
// eq. mom:sph:press:pij (asymm) or mom:sph:press:symm, then
// u^{n+1} = u* + dt f_p (eq. int:vnp1).
template <int KER, int D, typename R>
struct Correct {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.nf) return;
        Kern<KER, D, R> K(P.h);
        const int64_t nf = P.nf;
        const Pos xs = mkpos(S.xs);
        const double *p = S.p[0];
        double xi[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) xi[k] = xs.c[k][i];
        const double pi = p[i], rhoi_d = S.rho[i];
        const R rhoi = (R)rhoi_d, pi_r = (R)(pi / (rhoi_d * rhoi_d));
        R f[3] = {0, 0, 0};
        const int c = S.cnt[i];
        const bool symm = P.pgrad == SISPH_SYMM;
        if (sizeof(R) == 4 && symm) {
            // the 32-byte records: -m_j (p_i/rho_i^2 + p_j/rho_j^2) grad W
            const CorrRecS *srec = (const CorrRecS *)S.prec;
            for (int k0 = 1; k0 < c; k0 += kPairBatch) {
                int64_t jb[kPairBatch];
                batch_slots(S.nbr, nf, i, k0, c, P.cap, i, jb);
                CorrRecS rb[kPairBatch];
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) rb[t] = srec[jb[t]];
#pragma unroll
                for (int t = 0; t < kPairBatch; ++t) {
                    if (k0 + t >= c) break;
                    R d[3], r2;
                    pair_diff_v<D, R>(P.grid, xi, rb[t].x, d, r2);
                    const R dw = K.dwr(sqrt(r2));
                    R cf = -(R)rb[t].m * (pi_r + (R)rb[t].q);
                    cf *= dw;
                    for (int a = 0; a < D; ++a) f[a] += cf * d[a];
                }
            }
        }
        const CorrRec *crec = (const CorrRec *)S.prec;
        for (int k0 = 1; k0 < c && !(sizeof(R) == 4 && symm); k0 += kPairBatch) {
            int64_t jb[kPairBatch];
            double xj[kPairBatch][3], rhob[kPairBatch], pb[kPairBatch];
            R mb[kPairBatch];
            batch_slots(S.nbr, nf, i, k0, c, P.cap, i, jb);
            // one record per neighbour: r*, p, rho, m
            CorrRec rb[kPairBatch];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) rb[t] = crec[jb[t]];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                for (int a = 0; a < 3; ++a) xj[t][a] = rb[t].x[a];
                mb[t] = (R)rb[t].m;
                rhob[t] = rb[t].rho;
                pb[t] = rb[t].p;
            }
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                if (k0 + t >= c) break;
                R d[3], r2;
                pair_diff_v<D, R>(P.grid, xi, xj[t], d, r2);
                const R dw = K.dwr(sqrt(r2));
                const R mj = mb[t];
                const double rhoj = rhob[t];
                R cf;
                if (symm) cf = -mj * (pi_r + (R)(pb[t] / (rhoj * rhoj)));
                else cf = -mj / (rhoi * (R)rhoj) * (R)(pb[t] - pi);
                cf *= dw;
                for (int a = 0; a < D; ++a) f[a] += cf * d[a];
            }
        }
        const double dt = S.ctl->dt;
        for (int a = 0; a < D; ++a) {
            if (plain32(P)) {
                S.un[a][i] = (float)S.us[a][i] + (float)dt * (float)f[a];
                if (P.adaptive_dt) S.vk[a][i] = (float)S.vk[a][i] + (float)f[a];
            } else {
                S.un[a][i] = S.us[a][i] + dt * (double)f[a];
                if (P.adaptive_dt) S.vk[a][i] += (double)f[a];   // total acceleration of the step
            }
        }
    }
};

// Adaptive time step (section 3.2): the largest fluid speed at the start of
// the step (u still holds u^n here) and the largest total acceleration
// (predictor forces, gravity and pressure force, left in vk by the
// predictor and the correction), as squared magnitudes; non-negative
// doubles order like their bit patterns, so a wave max and one atomic max
// per wavefront give an order-independent result.
template <int D>
struct StepMaxima {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        if (!P.adaptive_dt) return;
        ROW;
        unsigned long long ub = 0ull, fb = 0ull;
        if (i < P.nf) {
#pragma clang fp contract(off)
            double u2 = 0.0, f2 = 0.0;
            for (int a = 0; a < D; ++a) {
                const double ua = S.u[a][i], fa = S.vk[a][i];
                u2 = u2 + ua * ua;
                f2 = f2 + fa * fa;
            }
            ub = (unsigned long long)__double_as_longlong(u2);
            fb = (unsigned long long)__double_as_longlong(f2);
        }
        ub = wave_max_u64(ub);
        fb = wave_max_u64(fb);
        if ((threadIdx.x & 63) == 0) {
            if (ub) max_if_larger(&S.ctl->umax2_bits, ub);
            if (fb) max_if_larger(&S.ctl->fmax2_bits, fb);
        }
    }
};

// dt^{n+1} = min(dt, 0.25 h / max|u^n|, 0.25 sqrt(h / max|f^n|)), the
// case's dt being the bound; a zero maximum imposes no limit.
struct NextDt {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t, int64_t, int) {
        if (threadIdx.x != 0 || !P.adaptive_dt) return;
        Control *c = S.ctl;
        const double u2 = __longlong_as_double((long long)c->umax2_bits);
        const double f2 = __longlong_as_double((long long)c->fmax2_bits);
        const double umax = sqrt(u2), fmax = sqrt(f2);
        double dt = P.dt;
        if (umax > 0.0 && 0.25 * P.h / umax < dt) dt = 0.25 * P.h / umax;
        if (fmax > 0.0 && 0.25 * sqrt(P.h / fmax) < dt) dt = 0.25 * sqrt(P.h / fmax);
        c->dt_next = rp(P, dt);
    }
};

// m_j / rho_j^2 of every particle in the working precision (the GTVF
// sub-steps read it per pair instead of m_j and rho_j), formed with the
// same operations the sub-steps used, so the values are identical.
template <typename R>
struct MassOverRho2 {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.ntot) return;
        const R rho = (R)S.rho[i];
        ((R *)S.mr2)[i] = (R)S.m[i] / (rho * rho);
    }
};

// --------------------------------------------------------- GTVF sub-steps
// The sub-steps gather a neighbour's position and m/rho^2 as one 32-byte
// record (two 16-byte loads instead of D + 1 scattered ones): the seed
// record of every particle at r* goes into gk[1], walls also into gk[0]
// (they never move); sub-step k reads gk[(k + 1) & 1] and writes its fluid
// rows into gk[k & 1].
template <typename R>
struct GtvfSeed {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.ntot || P.gtvf_K <= 0) return;
        const double4 r = make_double4(S.xs[0][i], P.dim > 1 ? S.xs[1][i] : 0.0, P.dim > 2 ? S.xs[2][i] : 0.0,
                                       (double)((const R *)S.mr2)[i]);
        S.gk[1][i] = r;
        if (i >= P.nf) S.gk[0][i] = r;
    }
};

// f = -p0_i sum_j m_j / rho_j^2 grad_i W(r_ij^{k-1}, h~) on the frozen r*
// neighbour lists (eq. mom:sph:gtvf), walls fixed;
// r^k = r^{k-1} + dtau u~^{k-1} + dtau^2/2 f, u~^k = u~^{k-1} + dtau f
// (eqs. int:gtvf:pos, int:gtvf:vel:tmp), no wrap inside the sub-steps.
template <int KER, int D, typename R>
struct Gtvf {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int k) {
        ROW;
        if (i >= P.nf || k >= P.gtvf_K) return;   // gtvf_K = 0 when GTVF is off
        const bool ext = P.gtvf == SISPH_GTVF_EXTERNAL;
        Kern<KER, D, R> K(ext ? 0.5 * P.h : P.h);
        const int64_t nf = P.nf;
        const double4 *src = S.gk[(k + 1) & 1];
        double4 *dst = S.gk[k & 1];
        const double4 own = src[i];
        const double xi[3] = {own.x, own.y, own.z};
        const double pref = S.ctl->p_ref;
        double p0 = pref;
        if (ext) {
            const double a = rp(P, 10.0 * fabs(S.p[0][i]));
            p0 = a < pref ? a : pref;
        }
        R s[3] = {0, 0, 0};
        // The short list while every particle is within sqrt(g_D2) of r*
        // (so far: sub-step k-1 raised g_disp_bits with r^{k-1} before this
        // launch; a raise by this launch can only select the full list):
        // a pair left out is then at least the support apart and adds
        // exactly zero, so the sum is the same bit for bit.
        const bool short_list = P.g_sub && !S.ctl->g_full &&
                                S.ctl->g_disp_bits <= (unsigned long long)__double_as_longlong(P.g_D2);
        const int32_t *list = short_list ? S.gnbr : S.nbr;
        const int k_first = short_list ? 0 : 1, c = short_list ? S.gcnt[i] : S.cnt[i];
        const int cap = short_list ? P.g_cap : P.cap;
        for (int k0 = k_first; k0 < c; k0 += kPairBatch) {
            int64_t jb[kPairBatch];
            double4 rb[kPairBatch];
            batch_slots(list, nf, i, k0, c, cap, i, jb);
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) rb[t] = src[jb[t]];
#pragma unroll
            for (int t = 0; t < kPairBatch; ++t) {
                if (k0 + t >= c) break;
                const double xj[3] = {rb[t].x, rb[t].y, rb[t].z};
                R d[3], r2;
                pair_diff_v<D, R>(P.grid, xi, xj, d, r2);
                const R dw = K.dwr(sqrt(r2));
                const R cf = (R)rb[t].w * dw;
                for (int a = 0; a < D; ++a) s[a] += cf * d[a];
            }
        }
        const double dtau = S.ctl->dt / (double)P.gtvf_K;
        double xn[3] = {xi[0], xi[1], xi[2]};
        for (int a = 0; a < D; ++a) {
            if (plain32(P)) {
                const float dtf = (float)dtau, f = -(float)p0 * (float)s[a];
                const float v = k == 0 ? 0.f : (float)S.vk[a][i];
                xn[a] = (float)xi[a] + dtf * v + 0.5f * dtf * dtf * f;
                S.vk[a][i] = v + dtf * f;
                continue;
            }
            const double f = -p0 * (double)s[a];
            const double v = k == 0 ? 0.0 : S.vk[a][i];
            xn[a] = xi[a] + dtau * v + 0.5 * dtau * dtau * f;
            S.vk[a][i] = v + dtau * f;
        }
        dst[i] = make_double4(xn[0], xn[1], xn[2], own.w);
        if (P.g_sub && k + 1 < P.gtvf_K) {
            // |r^k - r*|^2 (non-negative doubles order like their bits)
            double m2 = 0.0;
            for (int a = 0; a < D; ++a) {
                const double e = xn[a] - S.xs[a][i];
                m2 += e * e;
            }
            max_if_larger(&S.ctl->g_disp_bits, (unsigned long long)__double_as_longlong(m2));
        }
    }
};

// u~^{n+1} = u^{n+1} + (r^K - r^0)/dt (eq. int:vhatnp2);
// r^{n+1} = r^n + dt/2 (u~^{n+1} + u~^n) (eq. int:rnp2), wrapped.
// r^K is the last sub-step's buffer, or r* itself without GTVF.
template <int D>
struct Advance {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.nf) return;
        const int kfinal = P.gtvf_K - 1;
        double rk[3] = {0, 0, 0};
        if (kfinal < 0) {
            for (int a = 0; a < D; ++a) rk[a] = S.xs[a][i];
        } else {
            const double4 r = S.gk[kfinal & 1][i];
            rk[0] = r.x;
            rk[1] = r.y;
            rk[2] = r.z;
        }
        const double dt = S.ctl->dt;
        for (int a = 0; a < D; ++a) {
            double utn, xn;
            if (plain32(P)) {
                const float dtf = (float)dt;
                const float u1 = (float)S.un[a][i] + ((float)rk[a] - (float)S.xs[a][i]) / dtf;
                utn = u1;
                xn = (float)S.x[a][i] + 0.5f * dtf * (u1 + (float)S.ut[a][i]);
            } else {
                utn = S.un[a][i] + (rk[a] - S.xs[a][i]) / dt;
                xn = S.x[a][i] + 0.5 * dt * (utn + S.ut[a][i]);
            }
            S.x[a][i] = rp(P, wrap_periodic(xn, P.grid, a));
            S.ut[a][i] = utn;
            S.u[a][i] = S.un[a][i];
        }
    }
};

// -------------------------------------------------------------- BiCGStab
// The alternative PPE solver of section 3.1 on the cached coefficients:
// BiCGStab (van der Vorst 1992) on the system scaled by D_ii,
//   (M z)_i = z_i - sum_j c_ij z_j / D_ii,  f_i = (RHS_i + sum_w c_iw h_w) / D_ii
// on rows with D_ii != 0 off the free surface (z_i = 0 on the others), a
// wall neighbour's value being the linear part of eq. p-shepard applied to
// z and h_w its hydrostatic part (no clamp inside the solve).  Vectors and
// sums in FP64; the coefficients are the cached ones (FP32 in the mixed
// mode).  Iteration k runs as seven launches:
//   Dir (p = r + beta (p - omega v)), wall(p), MatV (v = M p, (r^, v)),
//   Step (alpha, s = r - alpha v), wall(s), MatT (t = M s, (t, s), (t, t)),
//   Update (omega, x += alpha p + omega s, r = s - omega t, (r^, r),
//   sum|r|, sum|x|).
// Scalars come from per-workgroup partial sums of an earlier launch, which
// every workgroup adds in the same order (so all agree), or from Control
// slots written by workgroup 0 of an earlier launch (slot k & 1, never the
// slot the current launch reads).  Dir of iteration k also takes the
// stopping decision after k-1 iterations in workgroup 0 (as the Jacobi
// sweep does); every later kernel of an iteration beyond the stop returns at
// once, so x keeps the final iterate.  A kernel tests stopped_at only
// against values that earlier launches write, so all its wavefronts agree.

enum { BP_RHO = 0, BP_ABSR, BP_ABSX, BP_RV, BP_TS, BP_TT, BP_ROWS };

__device__ __forceinline__ bool bicg_active(const State &S, int64_t i) { return S.dii[i] != 0.0 && !S.fs[i]; }

// Sum of one partial-sum row, in a fixed order, returned to every thread.
__device__ __forceinline__ double partial_total(const double *row, int64_t nblk) {
    __shared__ double sh[kBlock / 64];
    __shared__ double tot;
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < nblk; k += kBlock) a += row[k];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
        tot = t;
    }
    __syncthreads();
    return tot;
}

// Workgroup sum of v written to row[blk] (every thread must call).
__device__ __forceinline__ void partial_store(double v, double *row, int64_t blk) {
    __shared__ double sh[kBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
        row[blk] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ bool bicg_stopped(const State &S, int it) {
    return __hip_atomic_load(&S.ctl->stopped_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < it;
}

// (M z)_i for fluid row i (slot 0 is the particle itself, c_ii = 0).
template <typename R>
__device__ __forceinline__ double bicg_apply(const Params &P, const State &S, int64_t i, const double *z) {
    if (!bicg_active(S, i)) return z[i];
    const int64_t nf = P.nf;
    const int c = S.cnt[i];
    double acc = 0.0;
    for (int k = 1; k < c; ++k) {
        const int64_t at = group_at((k - 1) >> 2, nf, i) * 4 + ((k - 1) & 3);
        acc += (double)((const R *)S.coef)[at] * z[S.nbr[(int64_t)k * nf + i]];
    }
    return z[i] - acc / S.dii[i];
}

struct BicgInitX {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i < P.nf) S.bx[i] = bicg_active(S, i) ? S.p[0][i] : 0.0;
    }
};

// Wall slots of z (0: x, 1: p, 2: s) by the linear part of eq. p-shepard
// (the cached weights); with hydro, also the hydrostatic part h_w.
// it: the iteration (0 at set-up).
template <typename R>
struct BicgWall {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int, int which,
                                               int hydro, int it) {
        if (it > 0 && bicg_stopped(S, it)) return;
        ROW;
        if (i >= P.nw) return;
        double *z = which == 0 ? S.bx : (which == 1 ? S.bp : S.bs);
        const int64_t iw = P.nf + i, nw = P.nw;
        const int c = S.wcnt[i];
        double sz = 0.0;
        for (int k = 0; k < c; ++k) {
            const int64_t at = (int64_t)k * nw + i;
            if constexpr (sizeof(R) == 4) {
                const PairF e = ((const PairF *)S.wcoef)[(int64_t)S.woffw[i] + k];
                sz += (double)e.c * z[e.j];
            } else {
                sz += ((const double *)S.wcoef)[at] * z[S.wnbr[at]];
            }
        }
        z[iw] = sz;
        if (hydro) S.bh[iw] = S.wh[i];
    }
};

// f, r = f - M x, r^ = r, p = v = 0; partial (r^, r).
template <typename R>
struct BicgInitR {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int) {
        ROW;
        const int64_t nf = P.nf;
        double rr = 0.0;
        if (i < nf) {
            double f = 0.0, r = 0.0;
            if (bicg_active(S, i)) {
                double acc = 0.0;
                const int c = S.cnt[i];
                for (int k = 1; k < c; ++k) {
                    const int64_t j = S.nbr[(int64_t)k * nf + i];
                    const double cij = (double)((const R *)S.coef)[group_at((k - 1) >> 2, nf, i) * 4 + ((k - 1) & 3)];
                    if (j >= nf) acc += cij * S.bh[j];
                }
                f = (S.rhs[i] + acc) / S.dii[i];
                r = f - bicg_apply<R>(P, S, i, S.bx);
            }
            S.bf[i] = f;
            S.br[i] = r;
            S.brh[i] = r;
            S.bp[i] = 0.0;
            S.bv[i] = 0.0;
            rr = r * r;
        }
        partial_store(rr, S.bpart + BP_RHO * nblk, blk);
    }
};

// Iteration it: workgroup 0 first decides whether the solve stopped after
// it-1 iterations (eq. convergence on omega * sum|r| and sum|x|); then
// beta and the new direction p.
struct BicgDir {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int it) {
        // workgroup 0 of this launch may write stopped_at = it - 1, so only
        // a stop recorded by an earlier launch (below it - 1) is tested here
        if (bicg_stopped(S, it - 1)) return;
        Control *ctl = S.ctl;
        const double rho = partial_total(S.bpart + BP_RHO * nblk, nblk);
        if (blk == 0 && it >= 2) {
            __shared__ int stop_sh;
            const double num = P.omega * partial_total(S.bpart + BP_ABSR * nblk, nblk);
            const double den = partial_total(S.bpart + BP_ABSX * nblk, nblk);
            if (threadIdx.x == 0) {
                const int k = it - 1;
                double lam = __longlong_as_double((long long)ctl->lambda_bits);
                if (P.conv_norm == SISPH_CONV_MEAN) lam *= (double)P.nf;
                const double scale = lam > den ? lam : den;
                const double ratio = scale > 0.0 ? num / scale : (num > 0.0 ? INFINITY : 0.0);
                const bool bad = !isfinite(num) || !isfinite(den);
                bool stop = P.forced_iters > 0 ? k >= P.forced_iters : (ratio < P.tol || k >= P.max_iter);
                stop = stop || bad || ctl->bicg_brk;
                ctl->num = num;
                ctl->den = den;
                ctl->ratio = ratio;
                if (bad) ctl->nonfinite = 1;
                if (stop) {
                    ctl->iter = k;
                    ctl->done = 1;
                    ctl->stopped_at = k;
                }
                stop_sh = stop ? 1 : 0;
            }
            __syncthreads();
            if (stop_sh) return;
        }
        const int q = (it - 1) & 1;
        const double beta = (rho / ctl->bicg_rho[q]) * (ctl->bicg_alpha[q] / ctl->bicg_omega[q]);
        const double om = ctl->bicg_omega[q];
        ROW;
        if (i < P.nf) S.bp[i] = S.br[i] + beta * (S.bp[i] - om * S.bv[i]);
        if (blk == 0 && threadIdx.x == 0) ctl->bicg_rho[it & 1] = rho;
    }
};

// v = M p; partial (r^, v).
template <typename R>
struct BicgMatV {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int it) {
        if (bicg_stopped(S, it)) return;
        ROW;
        double a = 0.0;
        if (i < P.nf) {
            const double v = bicg_apply<R>(P, S, i, S.bp);
            S.bv[i] = v;
            a = S.brh[i] * v;
        }
        partial_store(a, S.bpart + BP_RV * nblk, blk);
    }
};

// alpha = rho / (r^, v); s = r - alpha v.
struct BicgStep {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int it) {
        if (bicg_stopped(S, it)) return;
        Control *ctl = S.ctl;
        const double rv = partial_total(S.bpart + BP_RV * nblk, nblk);
        const bool brk = rv == 0.0;
        const double alpha = brk ? 0.0 : ctl->bicg_rho[it & 1] / rv;
        ROW;
        if (i < P.nf) S.bs[i] = S.br[i] - alpha * S.bv[i];
        if (blk == 0 && threadIdx.x == 0) {
            ctl->bicg_alpha[it & 1] = alpha;
            if (brk) ctl->bicg_brk = 1;
        }
    }
};

// t = M s; partials (t, s), (t, t).
template <typename R>
struct BicgMatT {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int it) {
        if (bicg_stopped(S, it)) return;
        ROW;
        double ts = 0.0, tt = 0.0;
        if (i < P.nf) {
            const double t = bicg_apply<R>(P, S, i, S.bs);
            S.bt[i] = t;
            ts = t * S.bs[i];
            tt = t * t;
        }
        partial_store(ts, S.bpart + BP_TS * nblk, blk);
        partial_store(tt, S.bpart + BP_TT * nblk, blk);
    }
};

// omega = (t, s) / (t, t); x += alpha p + omega s; r = s - omega t;
// partials (r^, r), sum|r|, sum|x|.
struct BicgUpdate {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t nblk, int, int it) {
        if (bicg_stopped(S, it)) return;
        Control *ctl = S.ctl;
        const double ts = partial_total(S.bpart + BP_TS * nblk, nblk);
        const double tt = partial_total(S.bpart + BP_TT * nblk, nblk);
        const double om = tt == 0.0 ? 0.0 : ts / tt;
        const double alpha = ctl->bicg_alpha[it & 1];
        ROW;
        double rr = 0.0, ar = 0.0, ax = 0.0;
        if (i < P.nf) {
            const double x = S.bx[i] + alpha * S.bp[i] + om * S.bs[i];
            const double r = S.bs[i] - om * S.bt[i];
            S.bx[i] = x;
            S.br[i] = r;
            rr = S.brh[i] * r;
            ar = fabs(r);
            ax = fabs(x);
        }
        partial_store(rr, S.bpart + BP_RHO * nblk, blk);
        partial_store(ar, S.bpart + BP_ABSR * nblk, blk);
        partial_store(ax, S.bpart + BP_ABSX * nblk, blk);
        if (blk == 0 && threadIdx.x == 0) {
            ctl->bicg_omega[it & 1] = om;
            if (tt == 0.0) ctl->bicg_brk = 1;
            ctl->iter = it;
        }
    }
};

// x into p[0] and its FP32 copy (the final wall extrapolation of the mixed
// mode reads the copy).
struct BicgSettle {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i < P.nf) {
            const double x = S.bx[i];
            S.p[0][i] = x;
            S.p32[i] = (float)x;
        }
    }
};

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

}  // namespace

// ===================================================================== host
#define SISPH_DISPATCH_D(T, CALL)      \
    do {                               \
        if ((T).dim == 2) {            \
            constexpr int D = 2;       \
            CALL;                      \
        } else {                       \
            constexpr int D = 3;       \
            CALL;                      \
        }                              \
    } while (0)

#define SISPH_DISPATCH_KD(T, CALL)                         \
    do {                                                   \
        if ((T).kernel == SISPH_QUINTIC) {                 \
            constexpr int KER = SISPH_QUINTIC;             \
            SISPH_DISPATCH_D(T, CALL);                     \
        } else {                                           \
            constexpr int KER = SISPH_WENDLAND_C2;         \
            SISPH_DISPATCH_D(T, CALL);                     \
        }                                                  \
    } while (0)

#define SISPH_DISPATCH_KDR(T, CALL)                        \
    do {                                                   \
        if (f32_sums((T).precision)) {                     \
            using R = float;                               \
            SISPH_DISPATCH_KD(T, CALL);                    \
        } else {                                           \
            using R = double;                              \
            SISPH_DISPATCH_KD(T, CALL);                    \
        }                                                  \
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

__global__ __launch_bounds__(kBlock) void k_aos_to_soa(const double *__restrict__ src, double *d0, double *d1,
                                                       double *d2, int dim, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    d0[i] = src[i * dim];
    if (dim > 1) d1[i] = src[i * dim + 1];
    if (dim > 2) d2[i] = src[i * dim + 2];
}

// The plain FP32 mode starts from the case's state rounded to FP32:
// positions (fluid and walls), velocities, pressure and mass.
template <int D>
struct RoundState {
    static __device__ __forceinline__ void run(const Params &P, const State &S, int64_t blk, int64_t, int) {
        ROW;
        if (i >= P.ntot) return;
        for (int a = 0; a < D; ++a) {
            S.x[a][i] = (float)S.x[a][i];
            if (i < P.nf) {
                S.u[a][i] = (float)S.u[a][i];
                S.ut[a][i] = (float)S.ut[a][i];
            } else {
                S.wallu[a][i - P.nf] = (float)S.wallu[a][i - P.nf];
            }
        }
        S.p[0][i] = (float)S.p[0][i];
        S.m[i] = (float)S.m[i];
    }
};

void round_state(const Target &T) {
    if (T.precision == SISPH_FP32) SISPH_DISPATCH_D(T, (launch<RoundState<D>, K_TOT>(T)));
}

void aos_to_soa(const double *src, double *const dst[3], int64_t at, int dim, int64_t n, hipStream_t s) {
    if (n > 0)
        k_aos_to_soa<<<nblocks(n), kBlock, 0, s>>>(src, dst[0] + at, dim > 1 ? dst[1] + at : nullptr,
                                                    dim > 2 ? dst[2] + at : nullptr, dim, n);
}

void reset_control(const Target &T, int what) { launch<ResetControl, K_ONE>(T, what); }

void gather_control(const Target &T, Control *out) { launch<GatherControl, K_ONE>(T, out); }

void bin_fluid(const Target &T, int which) {
    launch<ZeroCount, K_CELL>(T);
    SISPH_DISPATCH_D(T, (launch<BinKeys<D>, K_FLUID>(T, which, 0)));
    launch<ScanTiles, K_TILE>(T, 0);
    launch<ScanSums, K_ONE>(T, 0);
    launch<ScanAdd, K_CELL>(T, 0);
    launch<Scatter, K_FLUID>(T, 0);
    launch<CellSort, K_CELLW>(T, 0, which == POS_X ? 1 : 0, which);
    if (which == POS_X) {
        SISPH_DISPATCH_D(T, (launch<ReorderFluid<D>, K_FLUID>(T, 0)));
        SISPH_DISPATCH_D(T, (launch<ReorderFluid<D>, K_FLUID>(T, 1)));
    } else {
        for (int batch = 0; batch < 2; ++batch) {
            SISPH_DISPATCH_D(T, (launch<ReorderStage2<D>, K_FLUID>(T, batch, 0)));
            SISPH_DISPATCH_D(T, (launch<ReorderStage2<D>, K_FLUID>(T, batch, 1)));
        }
    }
}

void bin_walls_once(const Target &T) {
    launch<ZeroCount, K_CELL>(T);
    SISPH_DISPATCH_D(T, (launch<BinKeys<D>, K_WALL>(T, (int)POS_X, 1)));
    launch<ScanTiles, K_TILE>(T, 1);
    launch<ScanSums, K_ONE>(T, 1);
    launch<ScanAdd, K_CELL>(T, 1);
    launch<Scatter, K_WALL>(T, 1);
    launch<CellSort, K_CELLW>(T, 1, 2, (int)POS_X);
    SISPH_DISPATCH_D(T, (launch<ReorderWalls<D>, K_WALL>(T, 0)));
    SISPH_DISPATCH_D(T, (launch<ReorderWalls<D>, K_WALL>(T, 1)));
}

void build_neighbors(const Target &T, int which) {
    // (without the density the kernel and precision do not enter: one instance per dimension)
    if (which == POS_X) SISPH_DISPATCH_KDR(T, (launch<BuildFluid<KER, D, R, true>, K_FLUID>(T, which)));
    else SISPH_DISPATCH_D(T, (launch<BuildFluid<SISPH_WENDLAND_C2, D, float, false>, K_FLUID>(T, which)));
    SISPH_DISPATCH_D(T, (launch<BuildWall<D>, K_WALL>(T, which)));
    // the sweeps read the lists at r* only
    if (which == POS_XS && T.packed) SISPH_DISPATCH_D(T, (launch<PackCodes<D>, K_FLUID>(T)));
}

void wall_normals(const Target &T) {
    SISPH_DISPATCH_KD(T, (launch<WallNormals<KER, D>, K_WALL>(T, 0)));
    SISPH_DISPATCH_KD(T, (launch<WallNormals<KER, D>, K_WALL>(T, 1)));
}

void wall_velocity(const Target &T, int which) {
    SISPH_DISPATCH_KDR(T, (launch<WallVelocity<KER, D, R>, K_WALL>(T, which)));
}

void predictor(const Target &T) { SISPH_DISPATCH_KDR(T, (launch<Predictor<KER, D, R>, K_FLUID>(T))); }

void rhs_coef(const Target &T) { SISPH_DISPATCH_KDR(T, (launch<RhsCoef<KER, D, R>, K_FLUID>(T))); }

void project_rhs(const Target &T) {
    launch<ProjectFinish, K_ONE>(T);
    launch<ProjectRhs, K_FLUID>(T);
}

void copy_p32(const Target &T) { launch<CopyP32, K_TOT>(T); }

// Sweep variants (numerically identical): first-batch size
// kSweepFirsts[v % kSweepFirstCount], XCD-contiguous workgroup mapping for
// v < kSweepFirstCount, hardware order otherwise.
template <typename R, bool PRE>
static void sweep_variant(const Target &T, int L, int v) {
    static_assert(kSweepFirstCount == 4 && kSweepVariants == 8, "one case per variant");
    switch (v) {
    case 1: launch<Sweep<R, kSweepFirsts[1], PRE>, K_FLUID, true>(T, L); break;
    case 2: launch<Sweep<R, kSweepFirsts[2], PRE>, K_FLUID, true>(T, L); break;
    case 3: launch<Sweep<R, kSweepFirsts[3], PRE>, K_FLUID, true>(T, L); break;
    case 4: launch<Sweep<R, kSweepFirsts[0], PRE>, K_FLUID, false>(T, L); break;
    case 5: launch<Sweep<R, kSweepFirsts[1], PRE>, K_FLUID, false>(T, L); break;
    case 6: launch<Sweep<R, kSweepFirsts[2], PRE>, K_FLUID, false>(T, L); break;
    case 7: launch<Sweep<R, kSweepFirsts[3], PRE>, K_FLUID, false>(T, L); break;
    default: launch<Sweep<R, kSweepFirsts[0], PRE>, K_FLUID, true>(T, L); break;
    }
}

void sweep_only(const Target &T, int L) {
    if (f32_sums(T.precision)) {
        if (T.precheck) sweep_variant<float, true>(T, L, T.variant);
        else sweep_variant<float, false>(T, L, T.variant);
    } else {
        if (T.precheck) sweep_variant<double, true>(T, L, T.variant);
        else sweep_variant<double, false>(T, L, T.variant);
    }
}

template <typename R, int FIRST>
static hipError_t persistent_launch(const Target &T, int limit) {
    const int64_t nb = kind_blocks(*T.P, K_FLUID);
    Params P = *T.P;
    State S = *T.S;
    void *args[] = {(void *)&P, (void *)&S, (void *)&limit};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_ppe_persistent<R, FIRST>), dim3((unsigned)nb),
                                      dim3(kBlock), args, 0, T.s);
}

template <typename R, int FIRST>
static int64_t persistent_capacity() {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_ppe_persistent<R, FIRST>),
                                                     kBlock, 0) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int64_t cap = (int64_t)per_cu * cus;
    return cap < (int64_t)kPartialRegs * kBlock ? cap : (int64_t)kPartialRegs * kBlock;
}

#define SISPH_PERSISTENT_FIRST(T, CALL)                                       \
    do {                                                                      \
        const int first = kSweepFirsts[(T).variant % kSweepFirstCount];       \
        if (f32_sums((T).precision)) {                                        \
            if (first <= 16) { using R = float; constexpr int F = 16; CALL; } \
            else if (first == 20) { using R = float; constexpr int F = 20; CALL; } \
            else { using R = float; constexpr int F = 24; CALL; }            \
        } else {                                                              \
            if (first <= 16) { using R = double; constexpr int F = 16; CALL; } \
            else if (first == 20) { using R = double; constexpr int F = 20; CALL; } \
            else { using R = double; constexpr int F = 24; CALL; }           \
        }                                                                     \
    } while (0)

hipError_t ppe_persistent(const Target &T, int limit) {
    SISPH_PERSISTENT_FIRST(T, return (persistent_launch<R, F>(T, limit)));
    return hipErrorInvalidValue;
}

int64_t ppe_persistent_capacity(const Target &T) {
    SISPH_PERSISTENT_FIRST(T, return (persistent_capacity<R, F>()));
    return 0;
}

template <typename R, int FIRST>
static hipError_t persistent_batch_launch(const Target &T, const int32_t *powner, const int64_t *pfirst,
                                          int64_t ptotal, uint32_t *bsync, int ncase, int limit, uint32_t spins) {
    const CaseEntry *tab = T.tab;
    void *args[] = {(void *)&tab, (void *)&powner, (void *)&pfirst, (void *)&bsync,
                    (void *)&ncase, (void *)&limit, (void *)&spins};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_ppe_persistent_batch<R, FIRST>),
                                      dim3((unsigned)ptotal), dim3(kBlock), args, 0, T.s);
}

template <typename R, int FIRST>
static int64_t persistent_batch_capacity() {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_ppe_persistent_batch<R, FIRST>), kBlock, 0) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int64_t cap = (int64_t)per_cu * cus;
    return cap < (int64_t)kPartialRegs * kBlock ? cap : (int64_t)kPartialRegs * kBlock;
}

hipError_t ppe_persistent_batch(const Target &T, const int32_t *powner, const int64_t *pfirst, int64_t ptotal,
                                uint32_t *bsync, int ncase, int limit, uint32_t spins) {
    SISPH_PERSISTENT_FIRST(T, return (persistent_batch_launch<R, F>(T, powner, pfirst, ptotal, bsync, ncase, limit,
                                                                     spins)));
    return hipErrorInvalidValue;
}

int64_t ppe_persistent_batch_capacity(const Target &T) {
    SISPH_PERSISTENT_FIRST(T, return (persistent_batch_capacity<R, F>()));
    return 0;
}

void ppe_iteration(const Target &T, int L) {
    if (T.solver == SISPH_BICGSTAB) {
        const int it = L + 1;
        launch<BicgDir, K_FLUID>(T, it);
        if (T.precision == SISPH_MIXED) launch<BicgWall<float>, K_WALL>(T, 1, 0, it);
        else launch<BicgWall<double>, K_WALL>(T, 1, 0, it);
        if (T.precision == SISPH_MIXED) launch<BicgMatV<float>, K_FLUID>(T, it);
        else launch<BicgMatV<double>, K_FLUID>(T, it);
        launch<BicgStep, K_FLUID>(T, it);
        if (T.precision == SISPH_MIXED) launch<BicgWall<float>, K_WALL>(T, 2, 0, it);
        else launch<BicgWall<double>, K_WALL>(T, 2, 0, it);
        if (T.precision == SISPH_MIXED) launch<BicgMatT<float>, K_FLUID>(T, it);
        else launch<BicgMatT<double>, K_FLUID>(T, it);
        launch<BicgUpdate, K_FLUID>(T, it);
        return;
    }
    wall_pressure_iteration(T, L);
    sweep_only(T, L);
}

void wall_pressure_iteration(const Target &T, int L) {
    // hardware workgroup order: the listed workgroups, which take the first
    // launch slots, then spread over every XCD
    if (f32_sums(T.precision)) launch<WallPressure<float>, K_WALLRUN, false>(T, L, 0);
    else launch<WallPressure<double>, K_WALL, false>(T, L, 0);
}

void bicg_begin(const Target &T) {
    launch<BicgInitX, K_FLUID>(T);
    if (T.precision == SISPH_MIXED) launch<BicgWall<float>, K_WALL>(T, 0, 1, 0);
    else launch<BicgWall<double>, K_WALL>(T, 0, 1, 0);
    if (T.precision == SISPH_MIXED) launch<BicgInitR<float>, K_FLUID>(T);
    else launch<BicgInitR<double>, K_FLUID>(T);
}

void bicg_settle(const Target &T) { launch<BicgSettle, K_FLUID>(T); }

void settle_pressure(const Target &T) { launch<SettlePressure, K_TOT>(T); }

void wall_pressure_final(const Target &T) {
    if (f32_sums(T.precision)) launch<WallPressure<float>, K_WALL>(T, 0, 1);
    else launch<WallPressure<double>, K_WALL>(T, 0, 1);
}

void wall_coef(const Target &T) {
    const bool walls = T.batched ? T.total[K_WALL] > 0 : kind_blocks(*T.P, K_WALL) > 0;
    if (!walls) return;
    launch<WallFlags, K_WALL>(T);
    launch<WallBlocks, K_ONE>(T);
    SISPH_DISPATCH_KDR(T, (launch<WallCoef<KER, D, R>, K_WALL>(T)));
}

void pressure_max(const Target &T) {
    launch<PMax, K_FLUID>(T);
    launch<PrefFinish, K_ONE>(T);
}

void correct(const Target &T) { SISPH_DISPATCH_KDR(T, (launch<Correct<KER, D, R>, K_FLUID>(T))); }

void step_maxima(const Target &T) { SISPH_DISPATCH_D(T, (launch<StepMaxima<D>, K_FLUID>(T))); }

void next_dt(const Target &T) { launch<NextDt, K_ONE>(T); }

void coef_seed(const Target &T) {
    if (f32_sums(T.precision)) launch<CoefSeed<float>, K_TOT>(T);
    else launch<CoefSeed<double>, K_TOT>(T);
}

void corr_seed(const Target &T) {
    if (f32_sums(T.precision)) launch<CorrSeed<float>, K_TOT>(T);
    else launch<CorrSeed<double>, K_TOT>(T);
}

void shadow(const Target &T) {
    if (f32_sums(T.precision)) launch<Shadow<float>, K_TOT>(T);
    else launch<Shadow<double>, K_TOT>(T);
}

void mass_over_rho2(const Target &T) {
    if (f32_sums(T.precision)) launch<MassOverRho2<float>, K_TOT>(T);
    else launch<MassOverRho2<double>, K_TOT>(T);
}

void gtvf_substep(const Target &T, int k) { SISPH_DISPATCH_KDR(T, (launch<Gtvf<KER, D, R>, K_FLUID>(T, k))); }

void gtvf_seed(const Target &T) {
    if (f32_sums(T.precision)) launch<GtvfSeed<float>, K_TOT>(T);
    else launch<GtvfSeed<double>, K_TOT>(T);
}

void advance(const Target &T) { SISPH_DISPATCH_D(T, (launch<Advance<D>, K_FLUID>(T))); }

}  // namespace sisph
