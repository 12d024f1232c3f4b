// Host runtime of libsisph: descriptor checks, workspace carving, the step
// state machine, batching and the C ABI declared in sisph.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sisph_internal.h"

using namespace sisph;

enum { ST_READY = 0, ST_BINNED = 1, ST_PREDICTED = 2, ST_SOLVED = 3 };

struct sisph_ctx {
    sisph_case_desc desc;
    Params P;
    State S;
    Target T;            // single-case launch target
    hipStream_t stream;
    int state;
    int nbr_stage;       // which neighbour lists are held: -1, 0 (r^n), 1 (r*)
    int last_iters;
    int prev_iters;   // the count before last_iters (0: none yet)
    Control *h_ctl;      // pinned mirror of the control block
    hipEvent_t ev[4];
    hipEvent_t evc[2];   // brackets one chunk of back-to-back sweeps
    double ppe_ms, step_ms;
    double sweep_ms;
    int64_t sweep_launches, sweep_effective;
    bool step_timed;
    bool step_pending = false;   // the last step's end event is recorded, its time not yet read
    bool ppe_pending = false;    // the same for the last solve (ev[1] .. ev[2])
    sisph_batch *batch;  // non-null while attached
    int32_t variant;     // Jacobi-sweep launch variant
    bool use_graphs = false;
    bool use_persistent = true;                                // one-launch solves where they apply
    int64_t persist_cap[kSweepFirstCount] = {-1, -1, -1, -1};                     // per first-batch size, -1: not asked yet
    int64_t persist_solves = 0;                                // since the counter reset
    int64_t persist_refused = 0, persist_timeouts = 0;         // fallbacks to per-launch sweeps
    int32_t persist_refusals[kSweepFirstCount] = {0, 0, 0, 0};   // per first-batch size, until it is given up
    bool persist_last = false;
    // sweep-kernel timing (sisph_set_kernel_timing): one event pair per
    // kt_period-th sweep launch of a chunk, the wall pass left out
    std::vector<hipEvent_t> kev;
    int32_t kt_period = 1;
    double kt_ms = 0.0;
    int64_t kt_launches = 0, kt_persistent = 0;
    bool is_static = false;                                    // lives in a device's static slot
    hipStream_t cap_stream = nullptr;                          // capture only
    hipGraphExec_t g_pre = nullptr, g_post = nullptr;          // fixed step segments
    std::string err;
};

static thread_local std::string g_create_err;
// sisph_create_static's last refusal (written without allocating)
static thread_local char g_static_err[256];
static thread_local bool g_static_err_set = false;

#define HIPCHK(ctx, expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
            return SISPH_E_DEVICE;                                                      \
        }                                                                               \
    } while (0)

// A context created in the static workspace has no events (creating them
// is an allocation): recording is skipped and its timings read zero.
static hipError_t ev_record(hipEvent_t e, hipStream_t s) { return e ? hipEventRecord(e, s) : hipSuccess; }
static hipError_t ev_elapsed(float *ms, hipEvent_t a, hipEvent_t b) {
    if (!a || !b) {
        *ms = 0.f;
        return hipSuccess;
    }
    return hipEventElapsedTime(ms, a, b);
}
static hipError_t ev_query(hipEvent_t e) { return e ? hipEventQuery(e) : hipSuccess; }
static hipError_t ev_sync(hipEvent_t e) { return e ? hipEventSynchronize(e) : hipSuccess; }

// ----------------------------------------------------------- descriptor
static double support_of(int kernel) { return kernel == SISPH_QUINTIC ? 3.0 : 2.0; }

static int32_t neighbour_cap(const sisph_case_desc *d);

static const char *check_desc(const sisph_case_desc *d) {
    if (!d) return "null descriptor";
    if (d->dim != 2 && d->dim != 3) return "dim must be 2 or 3";
    if (d->kernel != SISPH_QUINTIC && d->kernel != SISPH_WENDLAND_C2) return "unknown kernel";
    if (d->precision != SISPH_FP64 && d->precision != SISPH_MIXED && d->precision != SISPH_FP32)
        return "unknown precision";
    if (d->precision == SISPH_FP32 && d->solver != SISPH_JACOBI) return "the FP32 mode solves by Jacobi sweeps only";
    if (d->pgrad != SISPH_ASYMM && d->pgrad != SISPH_SYMM) return "unknown pressure-gradient form";
    if (d->gtvf < SISPH_GTVF_OFF || d->gtvf > SISPH_GTVF_EXTERNAL) return "unknown gtvf mode";
    if (d->p_ref_mode != SISPH_PREF_FIXED && d->p_ref_mode != SISPH_PREF_TWICE_MAX) return "unknown p_ref mode";
    if (d->conv_norm != SISPH_CONV_SUM && d->conv_norm != SISPH_CONV_MEAN) return "unknown conv_norm";
    if (d->ustar_wall != SISPH_USTAR_SLIP && d->ustar_wall != SISPH_USTAR_NOSLIP) return "unknown ustar_wall";
    if (d->dt_mode != SISPH_DT_FIXED && d->dt_mode != SISPH_DT_ADAPTIVE) return "unknown dt_mode";
    if (d->solver != SISPH_JACOBI && d->solver != SISPH_BICGSTAB) return "unknown solver";
    if (d->solver == SISPH_BICGSTAB && !d->free_surface)
        return "BiCGStab needs free-surface rows (otherwise p is fixed only up to a constant)";
    if (d->null_space != SISPH_NULL_NONE && d->null_space != SISPH_NULL_PROJECT) return "unknown null_space";
    if (d->null_space == SISPH_NULL_PROJECT && (d->n_wall != 0 || d->free_surface || d->solver != SISPH_JACOBI))
        return "null_space PROJECT needs a fully periodic Jacobi case (no walls, no free surface)";
    if (d->n_fluid <= 0) return "n_fluid must be positive";
    if (d->n_wall < 0) return "n_wall must be >= 0";
    if (d->n_fluid + d->n_wall >= (int64_t)1 << 31) return "particle count exceeds 2^31";
    if (!(d->h > 0) || !(d->dx > 0) || !(d->rho0 > 0) || !(d->dt > 0)) return "h, dx, rho0, dt must be positive";
    if (!(d->omega > 0) || !(d->omega <= 1.0)) return "omega must be in (0, 1]";
    if (d->min_iter < 1 || d->max_iter < d->min_iter) return "need 1 <= min_iter <= max_iter";
    if (d->max_iter >= INT32_MAX - 1) return "max_iter too large";
    if (d->forced_iters < 0 || d->forced_iters >= INT32_MAX - 1) return "forced_iters out of range";
    if (d->gtvf != SISPH_GTVF_OFF && d->gtvf_K < 1) return "gtvf_K must be >= 1";
    if (d->nbr_cap < 0) return "nbr_cap must be >= 0";
    if ((int64_t)neighbour_cap(d) * d->n_wall >= (int64_t)1 << 32)
        return "nbr_cap x n_wall reaches 2^32 (wall weight offsets are 32-bit)";
    double R = support_of(d->kernel) * d->h;
    for (int k = 0; k < d->dim; ++k) {
        double L = d->box_hi[k] - d->box_lo[k];
        if (!(L > 0)) return "box_hi must exceed box_lo";
        if (d->periodic[k] && L < 2.0 * R) return "a periodic axis must be at least two supports long";
    }
    return nullptr;
}

static Grid make_grid(const sisph_case_desc *d) {
    Grid g{};
    const double R = support_of(d->kernel) * d->h, Rm = R * 1.000001;
    g.ncell = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < d->dim) {
            g.lo[k] = d->box_lo[k];
            g.hi[k] = d->box_hi[k];
            g.L[k] = g.hi[k] - g.lo[k];
            g.Lh[k] = 0.5 * g.L[k];
            int64_t n = (int64_t)std::floor(g.L[k] / Rm);
            if (n < 1) n = 1;
            g.nc[k] = (int32_t)std::min<int64_t>(n, INT32_MAX);
            g.edge[k] = g.L[k] / (double)g.nc[k];
            if (g.edge[k] < Rm) g.edge[k] = Rm;
            g.per[k] = d->periodic[k] ? 1 : 0;
        } else {
            g.lo[k] = 0.0;
            g.hi[k] = 1.0;
            g.L[k] = 1.0;
            g.Lh[k] = 0.5;
            g.nc[k] = 1;
            g.edge[k] = 1.0;
            g.per[k] = 0;
        }
        g.ncell *= g.nc[k];
    }
    return g;
}

static int32_t neighbour_cap(const sisph_case_desc *d) {
    if (d->nbr_cap > 0) return (d->nbr_cap + 3) & ~3;   // whole groups of four slots
    const double R = support_of(d->kernel) * d->h / d->dx;
    const double pi = 3.14159265358979323846;
    double n = d->dim == 2 ? pi * R * R : 4.0 / 3.0 * pi * R * R * R;
    int32_t c = (int32_t)std::ceil(1.6 * n) + 8;
    return (c + 3) / 4 * 4;
}

static Params make_params(const sisph_case_desc *d) {
    Params P{};
    P.barrier_spins = kBarrierSpins;
    P.dim = d->dim;
    P.kernel = d->kernel;
    P.precision = d->precision;
    P.pgrad = d->pgrad;
    P.gtvf = d->gtvf;
    P.free_surface = d->free_surface ? 1 : 0;
    P.conv_norm = d->conv_norm;
    P.min_iter = d->min_iter;
    P.max_iter = d->max_iter;
    P.forced_iters = d->forced_iters;
    P.gtvf_K = d->gtvf == SISPH_GTVF_OFF ? 0 : d->gtvf_K;
    P.ustar_noslip = d->ustar_wall == SISPH_USTAR_NOSLIP ? 1 : 0;
    P.adaptive_dt = d->dt_mode == SISPH_DT_ADAPTIVE ? 1 : 0;
    P.solver = d->solver;
    P.null_space = d->null_space;
    P.compact = f32_sums(d->precision) && d->n_wall == 0 ? 1 : 0;
    P.packed = d->n_wall > 0 && !d->periodic[0] && d->solver == SISPH_JACOBI ? 1 : 0;
    P.cap = neighbour_cap(d);
    P.nf = d->n_fluid;
    P.nw = d->n_wall;
    P.ntot = d->n_fluid + d->n_wall;
    P.h = d->h;
    P.rho0 = d->rho0;
    P.nu = d->nu;
    P.alpha = d->alpha;
    P.c_ref = d->c_ref;
    P.dt = d->dt;
    P.eps_h = d->eta * d->h * d->h;
    P.fs_ratio = d->fs_ratio;
    P.omega = d->omega;
    P.tol = d->tol;
    const double R = support_of(d->kernel) * d->h;
    P.R2 = R * R;
    // GTVF short lists: the kernel support at h/2, widened by 1e-5 of it
    // (the FP32 kernel argument stays at or past the support for any pair
    // left out) and by twice the displacement bound (0.05 dx)
    P.g_sub = 0;
    P.g_cap = 0;
    P.g_R2 = 0.0;
    P.g_D2 = 0.0;
    if (d->gtvf == SISPH_GTVF_EXTERNAL && d->gtvf_K > 0) {
        const double dmax = 0.05 * d->dx, gR = support_of(d->kernel) * 0.5 * d->h * (1.0 + 1e-5) + 2.0 * dmax;
        if (gR < R) {
            const double q = gR / d->dx, pi = 3.14159265358979323846;
            const double n = d->dim == 2 ? pi * q * q : 4.0 / 3.0 * pi * q * q * q;
            P.g_sub = 1;
            P.g_cap = ((int32_t)std::ceil(1.6 * n) + 8 + 3) / 4 * 4;
            P.g_R2 = gR * gR;
            P.g_D2 = dmax * dmax;
        }
    }
    for (int k = 0; k < 3; ++k) P.g[k] = k < d->dim ? d->gravity[k] : 0.0;
    P.grid = make_grid(d);
    return P;
}

// ------------------------------------------------------------- workspace
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * (size_t)(count > 0 ? count : 1);
        return p;
    }
};

static void carve(const Params &P, Carver &c, State &S) {
    const int64_t nf = P.nf, nw = P.nw, nt = P.ntot, D = P.dim;
    auto vec = [&](double **dst, int64_t n) {
        for (int k = 0; k < 3; ++k) dst[k] = nullptr;
        for (int k = 0; k < D; ++k) dst[k] = c.take<double>(n);
    };
    vec(S.x, nt);
    vec(S.u, nt);
    vec(S.ut, nf);
    vec(S.xs, nt);
    vec(S.us, nt);
    vec(S.un, nf);
    S.gk[0] = c.take<double4>(nt);
    S.gk[1] = c.take<double4>(nt);
    S.gnbr = S.gcnt = nullptr;
    if (P.g_sub) {
        S.gnbr = c.take<int32_t>((int64_t)P.g_cap * nf);
        S.gcnt = c.take<int32_t>(nf);
    }
    vec(S.vk, nf);
    vec(S.nrm, nw);
    vec(S.wallu, nw);
    S.p[0] = c.take<double>(nt);
    S.p[1] = c.take<double>(nt);
    S.p32 = c.take<float>(2 * nt);
    S.m = c.take<double>(nt);
    S.rho = c.take<double>(nt);
    S.mr2 = c.take<double>(nt);
    S.m32 = S.rho32 = nullptr;
    if (f32_sums(P.precision)) {
        S.m32 = c.take<float>(nt);
        S.rho32 = c.take<float>(nt);
        S.prec = c.take<PredRecF>(nt);
    } else {
        S.prec = c.take<PredRecD>(nt);
    }
    S.rhs = c.take<double>(nf);
    S.dii = c.take<double>(nf);
    S.fs = c.take<int32_t>(nf);
    S.id = c.take<int32_t>(nf);
    S.wid = c.take<int32_t>(nw);
    const int64_t nmax = nf > nw ? nf : nw;
    S.key = c.take<uint32_t>(nmax);
    S.rank = c.take<uint32_t>(nmax);
    S.count = c.take<uint32_t>(P.grid.ncell);
    S.fstart = c.take<uint32_t>(P.grid.ncell + 1);
    S.wstart = c.take<uint32_t>(P.grid.ncell + 1);
    S.scan_tmp = c.take<uint32_t>(kind_blocks(P, K_TILE) + 1);
    S.perm = c.take<int32_t>(nmax);
    S.nbr = c.take<int32_t>((int64_t)P.cap * nf);
    S.cnt = c.take<int32_t>(nf);
    S.wnbr = c.take<int32_t>((int64_t)P.cap * nw);
    S.wcnt = c.take<int32_t>(nw);
    // mixed: (index, FP32 c_ij) 8-byte words; FP64: FP64 c_ij (indices from nbr)
    S.coef = c.take<char>((int64_t)8 * P.cap * nf);
    S.cidx = c.take<int32_t>((int64_t)P.cap * nf);
    S.pk12 = nullptr;
    S.stagerec = nullptr;
    S.rd32 = nullptr;
    S.cf = nullptr;
    if (P.packed) {
        S.pk12 = c.take<uint3>((int64_t)((P.cap + 6) / 8) * nf);
        S.stagerec = c.take<int32_t>(kind_blocks(P, K_FLUID) * kStageRec);
        if (f32_sums(P.precision)) {
            S.rd32 = c.take<float2>(nf);
            S.cf = c.take<int32_t>(nf);
        }
    }
    S.wcoef = c.take<char>((int64_t)8 * P.cap * nw);
    S.wh = c.take<double>(nw);
    S.wflag = c.take<int32_t>(kind_blocks(P, K_WALL) + 1);
    S.wblk = c.take<int32_t>(kind_blocks(P, K_WALL) + 1);
    S.wsum = c.take<uint32_t>(2 * kind_blocks(P, K_WALL) + 2);
    S.wrow = c.take<uint2>(nw + 1);
    S.woffw = c.take<uint32_t>(nw);
    S.partial = c.take<double>(4 * kind_blocks(P, K_FLUID));
    S.tmp = c.take<double>(16 * nmax);
    S.bx = S.br = S.brh = S.bp = S.bv = S.bs = S.bt = S.bf = S.bh = S.bpart = nullptr;
    if (P.solver == SISPH_BICGSTAB) {
        double **v[9] = {&S.bx, &S.br, &S.brh, &S.bp, &S.bv, &S.bs, &S.bt, &S.bf, &S.bh};
        for (auto *q : v) *q = c.take<double>(nt);
        S.bpart = c.take<double>(6 * kind_blocks(P, K_FLUID));
    }
    S.ctl = c.take<Control>(1);
    S.sync = c.take<uint32_t>(kSyncWords);
}

extern "C" size_t sisph_workspace_bytes(const sisph_case_desc *desc) {
    if (check_desc(desc)) return 0;
    Params P = make_params(desc);
    if (P.grid.ncell > ((int64_t)1 << 31) - 2) return 0;
    Carver c{nullptr};
    State S{};
    carve(P, c, S);
    return (c.off + 255) & ~(size_t)255;
}

static Target single_target(sisph_ctx *ctx) {
    Target T{};
    T.P = &ctx->P;
    T.S = &ctx->S;
    T.batched = false;
    T.ncase = 1;
    T.dim = ctx->P.dim;
    T.kernel = ctx->P.kernel;
    T.precision = ctx->P.precision;
    T.variant = ctx->variant;
    T.adaptive = ctx->P.adaptive_dt;
    T.packed = ctx->P.packed;
    T.precheck = ctx->P.nf >= kPrecheckRows ? 1 : 0;
    T.solver = ctx->P.solver;
    T.null_space = ctx->P.null_space;
    T.s = ctx->stream;
    return T;
}

// ------------------------------------------------------------ utilities
static int32_t h2d(sisph_ctx *ctx, double *dst, const double *src, int64_t n) {
    HIPCHK(ctx, hipMemcpyAsync(dst, src, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SISPH_OK;
}

// Host row-major [n][dim] -> device SoA component arrays (offset `at`),
// through the reorder scratch (16 x max(n_fluid, n_wall) doubles, free
// between steps) and a transpose kernel: no host staging buffer.
static int32_t upload_vec(sisph_ctx *ctx, double *const dst[3], int64_t at, const double *src, int64_t n) {
    const int D = ctx->P.dim;
    HIPCHK(ctx, hipMemcpyAsync(ctx->S.tmp, src, sizeof(double) * (size_t)(n * D), hipMemcpyHostToDevice,
                               ctx->stream));
    aos_to_soa(ctx->S.tmp, dst, at, D, n, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SISPH_OK;
}

static int32_t read_ctl(sisph_ctx *ctx) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_ctl, ctx->S.ctl, sizeof(Control), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SISPH_OK;
}

// The last step's time if its end has passed, else the previous value
// stays; done, without waiting, before the step's start event is recorded
// again.  A not-ready query is no error and is not left behind as one.
static void settle_step_time_if_done(sisph_ctx *ctx) {
    if (!ctx->step_pending) return;
    const hipError_t q = ev_query(ctx->ev[3]);
    if (q == hipSuccess) {
        float ms = 0.f;
        if (ev_elapsed(&ms, ctx->ev[0], ctx->ev[3]) == hipSuccess) ctx->step_ms = ms;
    } else if (q == hipErrorNotReady) {
        (void)hipGetLastError();
    }
    ctx->step_pending = false;
}

// The last solve's time, when the host did not wait for its end; done
// before its events are recorded again.
static int32_t settle_ppe_time(sisph_ctx *ctx) {
    if (!ctx->ppe_pending) return SISPH_OK;
    HIPCHK(ctx, ev_sync(ctx->ev[2]));
    float ms = 0.f;
    HIPCHK(ctx, ev_elapsed(&ms, ctx->ev[1], ctx->ev[2]));
    ctx->ppe_ms = ms;
    ctx->ppe_pending = false;
    return SISPH_OK;
}

static int32_t fail(sisph_ctx *ctx, int32_t code, const std::string &msg) {
    ctx->err = msg;
    return code;
}

static int32_t status_of(const Control &C, const Params &P, std::string *msg);

static void fill_stats(const Control &C, const Params &P, sisph_ppe_stats *out) {
    out->iters = C.iter;
    out->converged = C.ratio < P.tol ? 1 : 0;
    out->nonfinite = C.nonfinite;
    out->status = status_of(C, P, nullptr);
    out->ratio = C.ratio;
    union {
        unsigned long long u;
        double d;
    } cv;
    cv.u = C.lambda_bits;
    out->lambda = cv.d;
    out->p_ref = C.p_ref;
    out->dt = C.dt;
    out->index_bits = P.packed ? 12 : (P.compact && !C.wide ? 16 : 32);
    out->list_blocks = P.packed ? C.pk_overflow : 0;
    out->beta = P.null_space == SISPH_NULL_PROJECT ? C.beta : 0.0;
}

static int32_t status_of(const Control &C, const Params &P, std::string *msg) {
    if (C.overflow) {
        if (msg)
            *msg = "neighbour capacity exceeded: " + std::to_string(C.maxcnt) + " > nbr_cap " + std::to_string(P.cap);
        return SISPH_E_NOMEM;
    }
    if (C.nonfinite) {
        if (msg) *msg = "non-finite pressure in the PPE residual";
        return SISPH_E_NONFINITE;
    }
    if (P.forced_iters == 0 && !(C.ratio < P.tol)) return SISPH_WARN_MAXITER;
    return SISPH_OK;
}

// ---------------------------------------------------------------- create
// Sets a context up for a case whose workspace is carved already: uploads
// the state (through the workspace, no host buffers), clears the control
// block, bins the walls once and computes their normals.  On an error the
// message is in ctx->err.
static int32_t init_state(sisph_ctx *ctx, const sisph_case_desc *desc, const double *x, const double *u,
                          const double *p, const double *m, const double *wall_u) {
    auto fail_create = [](int32_t code) { return code; };
    {   // one mass for every particle (compared bit for bit)
        bool uni = ctx->P.ntot > 0;
        for (int64_t k = 1; uni && k < ctx->P.ntot; ++k) uni = std::memcmp(&m[k], &m[0], sizeof(double)) == 0;
        ctx->P.m_uni = uni ? 1 : 0;
        ctx->P.m_uni_f = uni ? (float)m[0] : 0.0f;
    }
    const Params &P = ctx->P;
    State &S = ctx->S;
    const int64_t nf = P.nf, nw = P.nw, nt = P.ntot, D = P.dim;
    hipStream_t s = ctx->stream;
    int32_t st;
    // state in caller order; fluid ids are 0..nf-1, wall ids 0..nw-1
    if ((st = upload_vec(ctx, S.x, 0, x, nt)) != SISPH_OK) return fail_create(st);
    if ((st = upload_vec(ctx, S.u, 0, u, nf)) != SISPH_OK) return fail_create(st);
    if ((st = upload_vec(ctx, S.ut, 0, u, nf)) != SISPH_OK) return fail_create(st);
    if ((st = h2d(ctx, S.p[0], p, nt)) != SISPH_OK) return fail_create(st);
    if ((st = h2d(ctx, S.m, m, nt)) != SISPH_OK) return fail_create(st);
    if (nw > 0) {
        if (wall_u) {
            if ((st = upload_vec(ctx, S.wallu, 0, wall_u, nw)) != SISPH_OK) return fail_create(st);
        } else {
            for (int k = 0; k < D; ++k) fill_f64(S.wallu[k], 0.0, nw, s);
        }
    }
    iota_i32(S.id, nf, s);
    iota_i32(S.wid, nw, s);
    round_state(ctx->T);
    reset_control(ctx->T, RESET_PPE | RESET_NEIGHBOURS | RESET_PREF | RESET_DT);
    if (desc->p_ref_mode == SISPH_PREF_FIXED) {
        Control c0{};
        c0.p_ref = desc->p_ref;
        c0.p_ref_set = 1;
        if (hipMemcpyAsync(&S.ctl->p_ref, &c0.p_ref, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(&S.ctl->p_ref_set, &c0.p_ref_set, sizeof(int32_t), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            ctx->err = "control upload failed";
            return fail_create(SISPH_E_DEVICE);
        }
    }
    // walls: one stable sort into cell order (they never move)
    fill_u32(S.wstart, 0u, P.grid.ncell + 1, s);
    if (nw > 0) {
        bin_walls_once(ctx->T);
        fill_f64(S.rho + nf, P.rho0, nw, s);
        fill_f64(S.p[0] + nf, 0.0, nw, s);
        fill_f64(S.p[1] + nf, 0.0, nw, s);
        for (int k = 0; k < D; ++k) {
            if (hipMemcpyAsync(S.xs[k] + nf, S.x[k] + nf, sizeof(double) * nw, hipMemcpyDeviceToDevice, s) !=
                hipSuccess) {
                ctx->err = "wall copy failed";
                return fail_create(SISPH_E_DEVICE);
            }
            fill_f64(S.u[k] + nf, 0.0, nw, s);
            fill_f64(S.us[k] + nf, 0.0, nw, s);
        }
        wall_normals(ctx->T);
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        ctx->err = "device error during create";
        return fail_create(SISPH_E_DEVICE);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char msg[200];
        std::snprintf(msg, sizeof msg, "kernel launch failed: %s", hipGetErrorString(e));
        ctx->err.assign(msg);
        return fail_create(SISPH_E_DEVICE);
    }
    return SISPH_OK;
}

// The host fields of a fresh context (everything but the workspace).
static void reset_ctx(sisph_ctx *ctx, const sisph_case_desc *desc, void *hip_stream) {
    ctx->desc = *desc;
    ctx->P = make_params(desc);
    ctx->stream = (hipStream_t)hip_stream;
    ctx->state = ST_READY;
    ctx->nbr_stage = -1;
    ctx->last_iters = desc->min_iter;
    ctx->prev_iters = 0;
    ctx->ppe_ms = ctx->step_ms = 0.0;
    ctx->sweep_ms = 0.0;
    ctx->sweep_launches = ctx->sweep_effective = 0;
    ctx->step_timed = false;
    ctx->step_pending = ctx->ppe_pending = false;
    ctx->batch = nullptr;
    ctx->variant = kDefaultVariant;
    ctx->use_graphs = false;
    ctx->use_persistent = true;
    for (auto &c : ctx->persist_cap) c = -1;
    ctx->persist_solves = ctx->persist_refused = ctx->persist_timeouts = 0;
    for (auto &r : ctx->persist_refusals) r = 0;
    ctx->persist_last = false;
    ctx->kt_ms = 0.0;
    ctx->kt_launches = ctx->kt_persistent = 0;
    ctx->err.clear();
}

// Descriptor, arrays and workspace size; the message of a refusal in *why.
static int32_t check_create(const sisph_case_desc *desc, const double *x, const double *u, const double *p,
                            const double *m, size_t *need, const char **why) {
    if ((*why = check_desc(desc))) return SISPH_E_INVAL;
    if (!x || !u || !p || !m) {
        *why = "null array argument";
        return SISPH_E_INVAL;
    }
    *need = sisph_workspace_bytes(desc);
    if (*need == 0) {
        *why = "binning grid too large";
        return SISPH_E_INVAL;
    }
    return SISPH_OK;
}

extern "C" int32_t sisph_create(const sisph_case_desc *desc, void *d_workspace, size_t ws_bytes, const double *x,
                                const double *u, const double *p, const double *m, const double *wall_u,
                                void *hip_stream, sisph_ctx **out) {
    if (!out) return SISPH_E_INVAL;
    *out = nullptr;
    g_static_err_set = false;
    size_t need = 0;
    const char *why = nullptr;
    int32_t st = check_create(desc, x, u, p, m, &need, &why);
    if (st != SISPH_OK) {
        g_create_err = why;
        return st;
    }
    if (!d_workspace) {
        g_create_err = "null workspace";
        return SISPH_E_INVAL;
    }
    if (((uintptr_t)d_workspace & 255) != 0) {
        g_create_err = "workspace must be 256-byte aligned";
        return SISPH_E_INVAL;
    }
    if (ws_bytes < need) {
        g_create_err = "workspace too small: need " + std::to_string(need) + " bytes";
        return SISPH_E_NOMEM;
    }
    sisph_ctx *ctx = new sisph_ctx();
    reset_ctx(ctx, desc, hip_stream);
    ctx->h_ctl = nullptr;
    for (auto &e : ctx->ev) e = nullptr;
    for (auto &e : ctx->evc) e = nullptr;
    Carver c{(char *)d_workspace};
    carve(ctx->P, c, ctx->S);
    ctx->T = single_target(ctx);
    auto bail = [&](int32_t code) {
        g_create_err = ctx->err;
        if (ctx->h_ctl) (void)hipHostFree(ctx->h_ctl);
        for (auto &e : ctx->ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : ctx->evc)
            if (e) (void)hipEventDestroy(e);
        delete ctx;
        return code;
    };
    if (hipHostMalloc((void **)&ctx->h_ctl, sizeof(Control), hipHostMallocDefault) != hipSuccess) {
        ctx->err = "hipHostMalloc failed";
        ctx->h_ctl = nullptr;
        return bail(SISPH_E_DEVICE);
    }
    for (auto &e : ctx->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            ctx->err = "hipEventCreate failed";
            return bail(SISPH_E_DEVICE);
        }
    for (auto &e : ctx->evc)
        if (hipEventCreate(&e) != hipSuccess) {
            ctx->err = "hipEventCreate failed";
            return bail(SISPH_E_DEVICE);
        }
    if ((st = init_state(ctx, desc, x, u, p, m, wall_u)) != SISPH_OK) return bail(st);
    *out = ctx;
    return SISPH_OK;
}

// ----------------------------------------------- the static workspace
// For callers that cannot allocate: one workspace per device in a
// file-scope device array.  In host code `scratch` names a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is used.  Each
// device also has one static host slot (the context and its control-block
// mirror in pageable memory), so a context created here allocates nothing:
// no device or pinned memory, no events (its timings read zero), no host
// heap.  A device holds one such context at a time.
static __device__ __align__(256) unsigned char scratch[SISPH_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
struct StaticSlot {
    void *ptr = nullptr;              // device address of scratch on this device
    std::atomic<int> in_use{0};
    sisph_ctx ctx;
    Control ctl;                      // host mirror of the control block
    StaticSlot() { ctx.err.reserve(512); }   // messages are written without allocating
};
StaticSlot g_static[kMaxDevices];
std::mutex g_static_mu;               // guards the one-time address lookups

int32_t static_refuse(int32_t code, const char *msg) {
    std::snprintf(g_static_err, sizeof g_static_err, "%s", msg);
    g_static_err_set = true;
    return code;
}
}  // namespace

extern "C" int32_t sisph_create_static(const sisph_case_desc *desc, const double *x, const double *u,
                                       const double *p, const double *m, const double *wall_u, void *hip_stream,
                                       sisph_ctx **out) {
    if (!out) return SISPH_E_INVAL;
    *out = nullptr;
    size_t need = 0;
    const char *why = nullptr;
    int32_t st = check_create(desc, x, u, p, m, &need, &why);
    if (st != SISPH_OK) return static_refuse(st, why);
    if (need > (size_t)SISPH_STATIC_WORKSPACE_BYTES) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "case needs %zu workspace bytes, above the static workspace's %zu", need,
                      (size_t)SISPH_STATIC_WORKSPACE_BYTES);
        return static_refuse(SISPH_E_NOMEM, msg);
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return static_refuse(SISPH_E_DEVICE, "no current device");
    StaticSlot &slot = g_static[dev];
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!slot.ptr) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) return static_refuse(SISPH_E_DEVICE, "hipGetSymbolAddress(scratch) failed");
            slot.ptr = ptr;
        }
    }
    int expect = 0;
    if (!slot.in_use.compare_exchange_strong(expect, 1))
        return static_refuse(SISPH_E_STATE, "the static workspace of this device holds a live context");
    sisph_ctx *ctx = &slot.ctx;
    reset_ctx(ctx, desc, hip_stream);
    ctx->is_static = true;
    ctx->h_ctl = &slot.ctl;
    for (auto &e : ctx->ev) e = nullptr;
    for (auto &e : ctx->evc) e = nullptr;
    Carver c{(char *)slot.ptr};
    carve(ctx->P, c, ctx->S);
    ctx->T = single_target(ctx);
    if ((st = init_state(ctx, desc, x, u, p, m, wall_u)) != SISPH_OK) {
        static_refuse(st, ctx->err.c_str());
        slot.in_use.store(0);
        return st;
    }
    g_static_err_set = false;
    *out = ctx;
    return SISPH_OK;
}

// Releases a context of the static workspace (called by sisph_destroy).
static void release_static(sisph_ctx *ctx) {
    for (auto &slot : g_static)
        if (&slot.ctx == ctx) slot.in_use.store(0);
}

// ------------------------------------------------------- step sequences
// The same launch sequences serve one case and a batch (Target).
static void seq_bin(const Target &T) {
    reset_control(T, RESET_NEIGHBOURS | RESET_STEP);
    bin_fluid(T, POS_X);
    build_neighbors(T, POS_X);
}

static void seq_predict(const Target &T) {
    // (the density and free-surface flag come from the build at r^n)
    mass_over_rho2(T);
    wall_velocity(T, POS_X);
    shadow(T);
    predictor(T);
    bin_fluid(T, POS_XS);
    build_neighbors(T, POS_XS);
    wall_velocity(T, POS_XS);
}

static void seq_ppe_begin(const Target &T) {
    reset_control(T, RESET_PPE);
    coef_seed(T);
    rhs_coef(T);
    if (T.null_space) project_rhs(T);
    wall_coef(T);
    if (T.solver == SISPH_BICGSTAB) bicg_begin(T);
    else if (f32_sums(T.precision)) copy_p32(T);
}

static void seq_ppe_end(const Target &T) {
    if (T.solver == SISPH_BICGSTAB) bicg_settle(T);
    else settle_pressure(T);
    wall_pressure_final(T);
    pressure_max(T);
}

static void seq_correct(const Target &T, int maxK) {
    corr_seed(T);
    correct(T);
    if (T.adaptive) {
        step_maxima(T);   // before the GTVF sub-steps reuse the acceleration buffer
        next_dt(T);
    }
    if (maxK > 0) gtvf_seed(T);
    for (int k = 0; k < maxK; ++k) gtvf_substep(T, k);
    advance(T);
}

// The fixed segments of a step around the data-dependent PPE loop: binning
// through the PPE set-up, and the settle through the advance.  They are
// captured once into graphs (kernel launches only: no copies or memsets)
// on a private stream and replayed on the caller's stream.
static void seq_pre(const Target &T) {
    seq_bin(T);
    seq_predict(T);
    seq_ppe_begin(T);
}

static void seq_post(const Target &T, int maxK) {
    seq_ppe_end(T);
    seq_correct(T, maxK);
}

template <class Seq>
static hipError_t capture_graph(hipStream_t &cs, Target T, Seq seq, hipGraphExec_t *out) {
    hipError_t e;
    if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return e;
    T.s = cs;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    seq(T);
    hipGraph_t g = nullptr;
    const hipError_t launched = hipGetLastError();
    e = hipStreamEndCapture(cs, &g);
    if (launched != hipSuccess) e = launched;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

static void drop_graphs(hipGraphExec_t &pre, hipGraphExec_t &post) {
    if (pre) (void)hipGraphExecDestroy(pre);
    if (post) (void)hipGraphExecDestroy(post);
    pre = post = nullptr;
}

// ------------------------------------------------------------ the stages
static bool attached(sisph_ctx *ctx) { return ctx->batch != nullptr; }

extern "C" int32_t sisph_bin(sisph_ctx *ctx) {
    if (!ctx) return SISPH_E_INVAL;
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    if (ctx->state != ST_READY) return fail(ctx, SISPH_E_STATE, "sisph_bin needs a completed step");
    settle_step_time_if_done(ctx);
    HIPCHK(ctx, ev_record(ctx->ev[0], ctx->stream));
    seq_bin(ctx->T);
    HIPCHK(ctx, hipGetLastError());
    ctx->state = ST_BINNED;
    ctx->nbr_stage = 0;
    ctx->step_timed = true;
    return SISPH_OK;
}

extern "C" int32_t sisph_predict(sisph_ctx *ctx) {
    if (!ctx) return SISPH_E_INVAL;
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    if (ctx->state != ST_BINNED) return fail(ctx, SISPH_E_STATE, "sisph_predict needs sisph_bin first");
    seq_predict(ctx->T);
    HIPCHK(ctx, hipGetLastError());
    ctx->state = ST_PREDICTED;
    ctx->nbr_stage = 1;
    return SISPH_OK;
}

// Sweeps to queue first for a case: the last solve's count moved on by its
// last change (counts drift slowly from step to step), unless that change
// was large (leaving the iteration limit, say); at least min_iter.  Only the
// launch count depends on it, never a result.
static int64_t predict_iters(const sisph_ctx *ctx) {
    const Params &P = ctx->P;
    if (P.forced_iters > 0) return P.forced_iters;
    int64_t p = ctx->last_iters;
    if (ctx->prev_iters > 0) {
        const int64_t trend = (int64_t)ctx->last_iters - ctx->prev_iters;
        if (8 * std::abs(trend) <= p) p += trend;
    }
    return std::max<int64_t>(p, P.min_iter);
}

static void record_iters(sisph_ctx *ctx, int iters) {
    ctx->prev_iters = ctx->last_iters;
    ctx->last_iters = std::max(iters, 1);
}

// Launch L performs sweep L unless its case stopped earlier; the decision
// for L sweeps is taken at the start of launch L, so each chunk of launches
// ends one beyond the predicted count.  poll() reads the control state and
// reports whether every case has stopped.
// Optional timing of the sweep kernel alone: each sweep launch of a chunk
// (up to the pool's size) between its own pair of events, read after the
// chunk's poll.
struct KTimer {
    hipEvent_t *ev;      // 2 per timed launch
    int64_t cap;         // timed launches the pool covers
    double *ms;
    int64_t *launches;
    int32_t period;      // every period-th launch of a solve (0, period, 2 period, ...)
};

template <class Poll>
static int32_t ppe_loop(const Target &T, int64_t predicted, int64_t limit, hipEvent_t e0, hipEvent_t e1,
                        double &sweep_ms, int64_t &launches, Poll poll, std::string &err,
                        const KTimer *kt = nullptr) {
    int64_t chunk = std::min<int64_t>(predicted + 1, limit);
    int64_t launched = 0;
    int polls = 0;
    for (;;) {
        if (ev_record(e0, T.s) != hipSuccess) return SISPH_E_DEVICE;
        int64_t timed = 0;
        for (int64_t c = 0; c < chunk; ++c) {
            if (kt && timed < kt->cap && T.solver == SISPH_JACOBI && (launched + c) % kt->period == 0) {
                wall_pressure_iteration(T, (int)(launched + c));
                if (hipEventRecord(kt->ev[2 * timed], T.s) != hipSuccess) return SISPH_E_DEVICE;
                sweep_only(T, (int)(launched + c));
                if (hipEventRecord(kt->ev[2 * timed + 1], T.s) != hipSuccess) return SISPH_E_DEVICE;
                ++timed;
            } else {
                ppe_iteration(T, (int)(launched + c));
            }
        }
        if (ev_record(e1, T.s) != hipSuccess) return SISPH_E_DEVICE;
        launched += chunk;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            err = std::string("sweep launch failed: ") + hipGetErrorString(e);
            return SISPH_E_DEVICE;
        }
        bool all_done = false;
        int32_t st = poll(all_done);
        if (st != SISPH_OK) return st;
        float cms = 0.f;
        if (ev_elapsed(&cms, e0, e1) != hipSuccess) return SISPH_E_DEVICE;
        sweep_ms += cms;
        launches += chunk;
        for (int64_t c = 0; c < timed; ++c) {
            float kms = 0.f;
            if (hipEventElapsedTime(&kms, kt->ev[2 * c], kt->ev[2 * c + 1]) != hipSuccess) return SISPH_E_DEVICE;
            *kt->ms += kms;
            *kt->launches += 1;
        }
        if (all_done || launched >= limit) break;
        // the prediction fell short: first by a little, as a rule (a
        // thirty-second of what has been launched), then grow by a quarter
        // of it (a launch past the stop is wasted, a poll costs a host
        // round trip)
        ++polls;
        const int64_t grow = polls == 1 ? launched / 32 : launched / 4;
        chunk = std::min<int64_t>(std::min<int64_t>(std::max<int64_t>(2, grow), 64), limit - launched);
        if (chunk < 1) chunk = 1;
    }
    return SISPH_OK;
}

// A case without walls, solved by Jacobi sweeps, whose fluid workgroups all
// fit on the device at once, runs its whole solve as one cooperative launch
// (ppe_persistent); other cases, or a launch the runtime refuses, take the
// per-launch sweeps.  Both give the same results and sweep counts.
constexpr int32_t kPersistRetries = 8;   // refused cooperative launches per first-batch size before giving up

static bool persistent_ok(sisph_ctx *ctx) {
    const Params &P = ctx->P;
    if (!ctx->use_persistent || P.nw > 0 || P.solver != SISPH_JACOBI) return false;
    const int64_t nb = kind_blocks(P, K_FLUID);
    int64_t &cap = ctx->persist_cap[ctx->T.variant % kSweepFirstCount];
    if (cap < 0) cap = ppe_persistent_capacity(ctx->T);
    return nb >= 1 && nb <= cap;
}

static int32_t ppe_run(sisph_ctx *ctx, int64_t predicted, int64_t limit) {
    ctx->persist_last = false;
    if (persistent_ok(ctx)) {
        // the starting iterate, kept in the binning scratch (unused during the
        // solve) in case the launch has to be redone with per-launch sweeps
        const size_t pbytes = sizeof(double) * (size_t)ctx->P.ntot;
        HIPCHK(ctx, hipMemcpyAsync(ctx->S.tmp, ctx->S.p[0], pbytes, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, ev_record(ctx->evc[0], ctx->stream));
        const hipError_t e = ppe_persistent(ctx->T, (int)limit);
        if (e == hipSuccess) {
            HIPCHK(ctx, ev_record(ctx->evc[1], ctx->stream));
            int32_t st = read_ctl(ctx);
            if (st != SISPH_OK) return st;
            if (ctx->h_ctl->barrier_late) {
                ctx->persist_timeouts += 1;
                // a workgroup never reached a barrier (the device was shared,
                // say): restore the starting iterate, set the solve up again
                // and run it with per-launch sweeps; this context keeps them
                for (auto &cap : ctx->persist_cap) cap = 0;
                HIPCHK(ctx, hipMemcpyAsync(ctx->S.p[0], ctx->S.tmp, pbytes, hipMemcpyDeviceToDevice, ctx->stream));
                seq_ppe_begin(ctx->T);
                HIPCHK(ctx, hipGetLastError());
                return ppe_run(ctx, predicted, limit);
            }
            float ms = 0.f;
            HIPCHK(ctx, ev_elapsed(&ms, ctx->evc[0], ctx->evc[1]));
            ctx->sweep_ms += ms;
            ctx->sweep_launches += ctx->h_ctl->iter + 1;   // sweeps run, the one after the stop included
            if (!ctx->kev.empty()) {   // the persistent launch is the sweep kernel
                ctx->kt_ms += ms;
                ctx->kt_launches += 1;
                ctx->kt_persistent += 1;
            }
            ctx->persist_solves += 1;
            ctx->persist_last = true;
            return SISPH_OK;
        }
        // refused (not all workgroups resident, say, or the device busy with
        // another process): this solve takes per-launch sweeps; the launch is
        // tried again on later solves, up to kPersistRetries refusals
        (void)hipGetLastError();
        ctx->persist_refused += 1;
        const int fi = ctx->T.variant % kSweepFirstCount;
        if (++ctx->persist_refusals[fi] >= kPersistRetries) ctx->persist_cap[fi] = 0;
    }
    auto poll = [&](bool &done) -> int32_t {
        int32_t st = read_ctl(ctx);
        if (st != SISPH_OK) return st;
        done = ctx->h_ctl->done != 0;
        return SISPH_OK;
    };
    KTimer kt{ctx->kev.data(), (int64_t)ctx->kev.size() / 2, &ctx->kt_ms, &ctx->kt_launches, ctx->kt_period};
    return ppe_loop(ctx->T, predicted, limit, ctx->evc[0], ctx->evc[1], ctx->sweep_ms, ctx->sweep_launches, poll,
                    ctx->err, ctx->kev.empty() ? nullptr : &kt);
}

extern "C" int32_t sisph_ppe_solve(sisph_ctx *ctx, sisph_ppe_stats *out) {
    if (!ctx) return SISPH_E_INVAL;
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    if (ctx->state != ST_PREDICTED) return fail(ctx, SISPH_E_STATE, "sisph_ppe_solve needs sisph_predict first");
    const Params &P = ctx->P;
    hipStream_t s = ctx->stream;
    int32_t st = settle_ppe_time(ctx);
    if (st != SISPH_OK) return st;
    HIPCHK(ctx, ev_record(ctx->ev[1], s));
    seq_ppe_begin(ctx->T);
    const int64_t limit = (int64_t)(P.forced_iters > 0 ? P.forced_iters : P.max_iter) + 1;
    const int64_t predicted = predict_iters(ctx);
    const int before = 0;
    st = ppe_run(ctx, predicted, limit);
    if (st != SISPH_OK) return st;
    // A persistent solve's control block, read at its end, already holds all
    // that the stats report once p_ref is set: the settle then only moves the
    // final iterate into buffer 0 (no walls, the maximum-pressure pass does
    // nothing), so the host does not wait for it and goes on queueing.
    const bool no_wait = ctx->persist_last && ctx->h_ctl->p_ref_set;
    seq_ppe_end(ctx->T);
    HIPCHK(ctx, ev_record(ctx->ev[2], s));
    if (no_wait) {
        HIPCHK(ctx, hipGetLastError());
        ctx->ppe_pending = true;
    } else {
        if ((st = read_ctl(ctx)) != SISPH_OK) return st;
        float ms = 0.f;
        HIPCHK(ctx, ev_elapsed(&ms, ctx->ev[1], ctx->ev[2]));
        ctx->ppe_ms = ms;
    }
    const Control &C = *ctx->h_ctl;
    ctx->sweep_effective += C.iter - before;
    record_iters(ctx, C.iter);
    if (out) fill_stats(C, P, out);
    ctx->state = ST_SOLVED;
    std::string msg;
    st = status_of(C, P, &msg);
    if (st < 0) return fail(ctx, st, msg);
    return st;
}

extern "C" int32_t sisph_correct(sisph_ctx *ctx) {
    if (!ctx) return SISPH_E_INVAL;
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    if (ctx->state != ST_SOLVED) return fail(ctx, SISPH_E_STATE, "sisph_correct needs sisph_ppe_solve first");
    hipStream_t s = ctx->stream;
    seq_correct(ctx->T, ctx->P.gtvf_K);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, ev_record(ctx->ev[3], s));
    ctx->step_pending = ctx->step_timed;   // read when asked: the host does not wait for the step here
    ctx->state = ST_READY;
    return SISPH_OK;
}

// One step with the fixed segments replayed from graphs.
static int32_t step_graphed(sisph_ctx *ctx, sisph_step_stats *out) {
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    if (ctx->state != ST_READY) return fail(ctx, SISPH_E_STATE, "sisph_step needs a completed step");
    const Params &P = ctx->P;
    hipStream_t s = ctx->stream;
    if (!ctx->g_pre) {
        hipError_t e = capture_graph(ctx->cap_stream, ctx->T, seq_pre, &ctx->g_pre);
        const int maxK = P.gtvf_K;
        if (e == hipSuccess)
            e = capture_graph(ctx->cap_stream, ctx->T, [maxK](const Target &T) { seq_post(T, maxK); },
                              &ctx->g_post);
        if (e != hipSuccess) {
            drop_graphs(ctx->g_pre, ctx->g_post);
            return fail(ctx, SISPH_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
    }
    const int32_t pst = settle_ppe_time(ctx);
    if (pst != SISPH_OK) return pst;
    settle_step_time_if_done(ctx);
    HIPCHK(ctx, ev_record(ctx->ev[0], s));
    HIPCHK(ctx, hipGraphLaunch(ctx->g_pre, s));
    HIPCHK(ctx, ev_record(ctx->ev[1], s));
    const int64_t limit = (int64_t)(P.forced_iters > 0 ? P.forced_iters : P.max_iter) + 1;
    const int64_t predicted = predict_iters(ctx);
    int32_t st = ppe_run(ctx, predicted, limit);
    if (st != SISPH_OK) return st;
    // as in sisph_ppe_solve: after a persistent solve with p_ref set, the
    // control block read at the solve's end is final for the stats
    const bool no_wait = ctx->persist_last && ctx->h_ctl->p_ref_set;
    HIPCHK(ctx, ev_record(ctx->ev[2], s));
    HIPCHK(ctx, hipGraphLaunch(ctx->g_post, s));
    HIPCHK(ctx, ev_record(ctx->ev[3], s));
    if (no_wait) {
        ctx->ppe_pending = true;   // the sweeps (set-up and settle are inside the graphs)
        ctx->step_pending = true;
    } else {
        if ((st = read_ctl(ctx)) != SISPH_OK) return st;
        float ms = 0.f;
        HIPCHK(ctx, ev_elapsed(&ms, ctx->ev[1], ctx->ev[2]));
        ctx->ppe_ms = ms;   // the sweeps (set-up and settle are inside the graphs)
        HIPCHK(ctx, ev_elapsed(&ms, ctx->ev[0], ctx->ev[3]));
        ctx->step_ms = ms;
        ctx->step_pending = false;
    }
    const Control &C = *ctx->h_ctl;
    ctx->sweep_effective += C.iter;
    record_iters(ctx, C.iter);
    ctx->nbr_stage = 1;
    if (out) fill_stats(C, P, out);
    ctx->state = ST_READY;
    std::string msg;
    st = status_of(C, P, &msg);
    if (st < 0) return fail(ctx, st, msg);
    return st;
}

extern "C" int32_t sisph_step(sisph_ctx *ctx, int32_t nsteps, sisph_step_stats *out) {
    if (!ctx || nsteps < 0) return SISPH_E_INVAL;
    int32_t worst = SISPH_OK;
    if (ctx->use_graphs) {
        for (int32_t n = 0; n < nsteps; ++n) {
            const int32_t sp = step_graphed(ctx, out ? out + n : nullptr);
            if (sp < 0) return sp;
            if (sp > worst) worst = sp;
        }
        return worst;
    }
    for (int32_t n = 0; n < nsteps; ++n) {
        int32_t st = sisph_bin(ctx);
        if (st < 0) return st;
        if ((st = sisph_predict(ctx)) < 0) return st;
        int32_t sp = sisph_ppe_solve(ctx, out ? out + n : nullptr);
        if (sp < 0) return sp;
        if ((st = sisph_correct(ctx)) < 0) return st;
        if (sp > worst) worst = sp;
    }
    return worst;
}

// --------------------------------------------------------- state access
template <typename T>
static int32_t d2h(sisph_ctx *ctx, std::vector<T> &dst, const T *src, int64_t n) {
    dst.resize((size_t)(n > 0 ? n : 0));
    if (n <= 0) return SISPH_OK;
    HIPCHK(ctx, hipMemcpyAsync(dst.data(), src, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SISPH_OK;
}

// Device SoA (sorted) -> host row-major in original order via the id map.
static int32_t download_vec(sisph_ctx *ctx, double *dst, double *const src[3], int64_t at, int64_t n,
                            const std::vector<int32_t> &ids, int64_t dst_off) {
    const int D = ctx->P.dim;
    std::vector<double> col;
    for (int k = 0; k < D; ++k) {
        int32_t st = d2h(ctx, col, src[k] + at, n);
        if (st != SISPH_OK) return st;
        for (int64_t i = 0; i < n; ++i) dst[(dst_off + ids[(size_t)i]) * D + k] = col[(size_t)i];
    }
    return SISPH_OK;
}

static int32_t download_scalar(sisph_ctx *ctx, double *dst, const double *src, int64_t n,
                               const std::vector<int32_t> &ids, int64_t dst_off) {
    std::vector<double> col;
    int32_t st = d2h(ctx, col, src, n);
    if (st != SISPH_OK) return st;
    for (int64_t i = 0; i < n; ++i) dst[dst_off + ids[(size_t)i]] = col[(size_t)i];
    return SISPH_OK;
}

extern "C" int32_t sisph_read_state(sisph_ctx *ctx, double *x, double *u, double *u_tilde, double *p,
                                    double *rho) {
    if (!ctx) return SISPH_E_INVAL;
    if (ctx->state != ST_READY && ctx->state != ST_BINNED)
        return fail(ctx, SISPH_E_STATE, "state is readable between steps only");
    const Params &P = ctx->P;
    State &S = ctx->S;
    std::vector<int32_t> id, wid;
    int32_t st;
    if ((st = d2h(ctx, id, S.id, P.nf)) != SISPH_OK) return st;
    if ((st = d2h(ctx, wid, S.wid, P.nw)) != SISPH_OK) return st;
    if (x) {
        if ((st = download_vec(ctx, x, S.x, 0, P.nf, id, 0)) != SISPH_OK) return st;
        if (P.nw && (st = download_vec(ctx, x, S.x, P.nf, P.nw, wid, P.nf)) != SISPH_OK) return st;
    }
    if (u && (st = download_vec(ctx, u, S.u, 0, P.nf, id, 0)) != SISPH_OK) return st;
    if (u_tilde && (st = download_vec(ctx, u_tilde, S.ut, 0, P.nf, id, 0)) != SISPH_OK) return st;
    if (p) {
        if ((st = download_scalar(ctx, p, S.p[0], P.nf, id, 0)) != SISPH_OK) return st;
        if (P.nw && (st = download_scalar(ctx, p, S.p[0] + P.nf, P.nw, wid, P.nf)) != SISPH_OK) return st;
    }
    if (rho && (st = download_scalar(ctx, rho, S.rho, P.nf, id, 0)) != SISPH_OK) return st;
    return SISPH_OK;
}

extern "C" int32_t sisph_write_state(sisph_ctx *ctx, const double *x, const double *u, const double *u_tilde,
                                     const double *p) {
    if (!ctx) return SISPH_E_INVAL;
    if (ctx->state != ST_READY) return fail(ctx, SISPH_E_STATE, "state is writable between steps only");
    const Params &P = ctx->P;
    State &S = ctx->S;
    const int D = P.dim;
    std::vector<int32_t> id;
    int32_t st;
    if ((st = d2h(ctx, id, S.id, P.nf)) != SISPH_OK) return st;
    // write in the current sorted order so that fields stay aligned
    auto put_vec = [&](double *const dst[3], const double *src) -> int32_t {
        std::vector<double> col((size_t)P.nf);
        for (int k = 0; k < D; ++k) {
            for (int64_t i = 0; i < P.nf; ++i) col[(size_t)i] = src[(int64_t)id[(size_t)i] * D + k];
            HIPCHK(ctx, hipMemcpyAsync(dst[k], col.data(), sizeof(double) * (size_t)P.nf, hipMemcpyHostToDevice,
                                       ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        }
        return SISPH_OK;
    };
    if (x && (st = put_vec(S.x, x)) != SISPH_OK) return st;
    if (u && (st = put_vec(S.u, u)) != SISPH_OK) return st;
    if (u_tilde && (st = put_vec(S.ut, u_tilde)) != SISPH_OK) return st;
    if (p) {
        std::vector<double> col((size_t)P.nf);
        for (int64_t i = 0; i < P.nf; ++i) col[(size_t)i] = p[id[(size_t)i]];
        HIPCHK(ctx, hipMemcpyAsync(S.p[0], col.data(), sizeof(double) * (size_t)P.nf, hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return SISPH_OK;
}

extern "C" int32_t sisph_read_field(sisph_ctx *ctx, int32_t field, double *out) {
    if (!ctx || !out) return SISPH_E_INVAL;
    const Params &P = ctx->P;
    State &S = ctx->S;
    std::vector<int32_t> id, wid;
    int32_t st;
    if ((st = d2h(ctx, id, S.id, P.nf)) != SISPH_OK) return st;
    if ((st = d2h(ctx, wid, S.wid, P.nw)) != SISPH_OK) return st;
    switch (field) {
    case SISPH_FIELD_RHO: return download_scalar(ctx, out, S.rho, P.nf, id, 0);
    case SISPH_FIELD_XSTAR: return download_vec(ctx, out, S.xs, 0, P.nf, id, 0);
    case SISPH_FIELD_USTAR: return download_vec(ctx, out, S.us, 0, P.nf, id, 0);
    case SISPH_FIELD_RHS: return download_scalar(ctx, out, S.rhs, P.nf, id, 0);
    case SISPH_FIELD_DII: return download_scalar(ctx, out, S.dii, P.nf, id, 0);
    case SISPH_FIELD_UNEW: return download_vec(ctx, out, S.un, 0, P.nf, id, 0);
    case SISPH_FIELD_WALL_U: return download_vec(ctx, out, S.u, P.nf, P.nw, wid, 0);
    case SISPH_FIELD_WALL_USTAR: return download_vec(ctx, out, S.us, P.nf, P.nw, wid, 0);
    case SISPH_FIELD_NORMAL: return download_vec(ctx, out, S.nrm, 0, P.nw, wid, 0);
    case SISPH_FIELD_FS: {
        std::vector<int32_t> f;
        if ((st = d2h(ctx, f, S.fs, P.nf)) != SISPH_OK) return st;
        for (int64_t i = 0; i < P.nf; ++i) out[id[(size_t)i]] = (double)f[(size_t)i];
        return SISPH_OK;
    }
    case SISPH_FIELD_PRESSURE: {
        if ((st = download_scalar(ctx, out, S.p[0], P.nf, id, 0)) != SISPH_OK) return st;
        if (P.nw) return download_scalar(ctx, out, S.p[0] + P.nf, P.nw, wid, P.nf);
        return SISPH_OK;
    }
    default: return fail(ctx, SISPH_E_INVAL, "unknown field");
    }
}

extern "C" int32_t sisph_pair_count(sisph_ctx *ctx, int32_t stage, int32_t dest, int64_t *pairs) {
    if (!ctx || !pairs || (dest != 0 && dest != 1)) return SISPH_E_INVAL;
    if (stage != ctx->nbr_stage) return fail(ctx, SISPH_E_STATE, "requested neighbour stage is not held");
    int32_t st = read_ctl(ctx);
    if (st != SISPH_OK) return st;
    if (ctx->h_ctl->overflow)
        return fail(ctx, SISPH_E_NOMEM, "neighbour capacity exceeded: " + std::to_string(ctx->h_ctl->maxcnt));
    std::vector<int32_t> cnt;
    const int64_t rows = dest == 0 ? ctx->P.nf : ctx->P.nw;
    if ((st = d2h(ctx, cnt, dest == 0 ? ctx->S.cnt : ctx->S.wcnt, rows)) != SISPH_OK) return st;
    int64_t tot = 0;
    for (int32_t c : cnt) tot += c;
    *pairs = tot;
    return SISPH_OK;
}

extern "C" int32_t sisph_rows_with_neighbours(sisph_ctx *ctx, int32_t stage, int32_t dest, int64_t *rows) {
    if (!ctx || !rows || (dest != 0 && dest != 1)) return SISPH_E_INVAL;
    if (stage != ctx->nbr_stage) return fail(ctx, SISPH_E_STATE, "requested neighbour stage is not held");
    int32_t st = read_ctl(ctx);
    if (st != SISPH_OK) return st;
    if (ctx->h_ctl->overflow)
        return fail(ctx, SISPH_E_NOMEM, "neighbour capacity exceeded: " + std::to_string(ctx->h_ctl->maxcnt));
    std::vector<int32_t> cnt;
    const int64_t n = dest == 0 ? ctx->P.nf : ctx->P.nw;
    if ((st = d2h(ctx, cnt, dest == 0 ? ctx->S.cnt : ctx->S.wcnt, n)) != SISPH_OK) return st;
    const int32_t self = dest == 0 ? 1 : 0;   // fluid lists hold the row itself first
    int64_t tot = 0;
    for (int32_t c : cnt) tot += c > self;
    *rows = tot;
    return SISPH_OK;
}

extern "C" int32_t sisph_debug_neighbors(sisph_ctx *ctx, int32_t stage, int32_t dest, int64_t *offsets,
                                         int32_t *ids, int64_t cap) {
    if (!ctx || !offsets || (dest != 0 && dest != 1)) return SISPH_E_INVAL;
    if (stage != ctx->nbr_stage) return fail(ctx, SISPH_E_STATE, "requested neighbour stage is not held");
    const Params &P = ctx->P;
    State &S = ctx->S;
    int32_t st = read_ctl(ctx);
    if (st != SISPH_OK) return st;
    if (ctx->h_ctl->overflow)
        return fail(ctx, SISPH_E_NOMEM, "neighbour capacity exceeded: " + std::to_string(ctx->h_ctl->maxcnt));
    std::vector<int32_t> id, wid, nbr, cnt;
    if ((st = d2h(ctx, id, S.id, P.nf)) != SISPH_OK) return st;
    if ((st = d2h(ctx, wid, S.wid, P.nw)) != SISPH_OK) return st;
    const int64_t rows = dest == 0 ? P.nf : P.nw;
    if ((st = d2h(ctx, nbr, dest == 0 ? S.nbr : S.wnbr, (int64_t)P.cap * rows)) != SISPH_OK) return st;
    if ((st = d2h(ctx, cnt, dest == 0 ? S.cnt : S.wcnt, rows)) != SISPH_OK) return st;
    auto orig = [&](int64_t j) -> int32_t {
        return j < P.nf ? id[(size_t)j] : (int32_t)(P.nf + wid[(size_t)(j - P.nf)]);
    };
    std::vector<std::vector<int32_t>> out((size_t)rows);
    for (int64_t r = 0; r < rows; ++r) {
        int64_t orow = dest == 0 ? id[(size_t)r] : wid[(size_t)r];
        auto &v = out[(size_t)orow];
        for (int k = 0; k < cnt[(size_t)r]; ++k) v.push_back(orig(nbr[(size_t)((int64_t)k * rows + r)]));
        std::sort(v.begin(), v.end());
    }
    int64_t tot = 0;
    offsets[0] = 0;
    for (int64_t r = 0; r < rows; ++r) {
        for (int32_t j : out[(size_t)r]) {
            if (tot < cap && ids) ids[tot] = j;
            ++tot;
        }
        offsets[r + 1] = tot;
    }
    if (tot > cap) return fail(ctx, SISPH_E_NOMEM, "ids buffer too small");
    return SISPH_OK;
}

extern "C" int32_t sisph_last_timings(sisph_ctx *ctx, double *ppe_ms, double *step_ms) {
    if (!ctx) return SISPH_E_INVAL;
    const int32_t st = settle_ppe_time(ctx);
    if (st != SISPH_OK) return st;
    if (ctx->step_pending) {
        HIPCHK(ctx, ev_sync(ctx->ev[3]));
        float ms = 0.f;
        HIPCHK(ctx, ev_elapsed(&ms, ctx->ev[0], ctx->ev[3]));
        ctx->step_ms = ms;
        ctx->step_pending = false;
    }
    if (ppe_ms) *ppe_ms = ctx->ppe_ms;
    if (step_ms) *step_ms = ctx->step_ms;
    return SISPH_OK;
}

extern "C" int32_t sisph_sweep_counters(sisph_ctx *ctx, double *sweep_ms, int64_t *launches, int64_t *effective,
                                        int32_t reset) {
    if (!ctx) return SISPH_E_INVAL;
    if (sweep_ms) *sweep_ms = ctx->sweep_ms;
    if (launches) *launches = ctx->sweep_launches;
    if (effective) *effective = ctx->sweep_effective;
    if (reset) {
        ctx->sweep_ms = 0.0;
        ctx->sweep_launches = ctx->sweep_effective = 0;
        ctx->persist_solves = 0;
        ctx->persist_refused = ctx->persist_timeouts = 0;
        ctx->kt_ms = 0.0;
        ctx->kt_launches = ctx->kt_persistent = 0;
    }
    return SISPH_OK;
}

extern "C" int32_t sisph_set_kernel_timing(sisph_ctx *ctx, int32_t period) {
    if (!ctx) return SISPH_E_INVAL;
    if (period <= 0) {
        for (auto &e : ctx->kev) (void)hipEventDestroy(e);
        ctx->kev.clear();
        return SISPH_OK;
    }
    if (ctx->is_static) return fail(ctx, SISPH_E_STATE, "a context in the static workspace creates no events");
    ctx->kt_period = period;
    if (!ctx->kev.empty()) return SISPH_OK;
    // one pair per launch a chunk can hold: max_iter + 1 (or forced_iters + 1)
    const int64_t n = 2 * ((int64_t)(ctx->P.forced_iters > 0 ? ctx->P.forced_iters : ctx->P.max_iter) + 1);
    ctx->kev.assign((size_t)n, nullptr);
    for (auto &e : ctx->kev) {
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ctx->kev)
                if (f) (void)hipEventDestroy(f);
            ctx->kev.clear();
            return fail(ctx, SISPH_E_DEVICE, "hipEventCreate failed");
        }
    }
    return SISPH_OK;
}

extern "C" int32_t sisph_kernel_timing(sisph_ctx *ctx, double *ms, int64_t *launches, int64_t *persistent) {
    if (!ctx) return SISPH_E_INVAL;
    if (ms) *ms = ctx->kt_ms;
    if (launches) *launches = ctx->kt_launches;
    if (persistent) *persistent = ctx->kt_persistent;
    return SISPH_OK;
}

extern "C" int32_t sisph_debug_barrier_spins(sisph_ctx *ctx, uint32_t spins) {
    if (!ctx) return SISPH_E_INVAL;
    ctx->P.barrier_spins = spins;
    return SISPH_OK;
}

extern "C" int32_t sisph_debug_packed(sisph_ctx *ctx, int32_t on) {
    if (!ctx) return SISPH_E_INVAL;
    const bool can = make_params(&ctx->desc).packed != 0;   // its buffers exist
    if (on && !can) return fail(ctx, SISPH_E_INVAL, "this case has no packed mode");
    ctx->P.packed = on && can ? 1 : 0;
    ctx->T = single_target(ctx);
    drop_graphs(ctx->g_pre, ctx->g_post);   // captured with the old parameters
    return SISPH_OK;
}

// Read-rate probe: 16-byte loads, grid-stride, four in flight per thread,
// one float sum per thread (so no load is dead).
__global__ __launch_bounds__(kBlock) void k_read_rate(const float4 *__restrict__ a, int64_t n4, float *out) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float s = 0.0f;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
        s += (v0.x + v0.y + v0.z + v0.w) + (v1.x + v1.y + v1.z + v1.w) + (v2.x + v2.y + v2.z + v2.w) +
             (v3.x + v3.y + v3.z + v3.w);
    }
    for (; i < n4; i += stride) {
        const float4 v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

extern "C" int32_t sisph_debug_read_rate(const void *buf, int64_t bytes, float *out, int32_t grid, int32_t reps,
                                         double *us) {
    if (!buf || !out || !us || bytes <= 0 || bytes % 16 != 0 || grid < 1 || reps < 1) return SISPH_E_INVAL;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int64_t n4 = bytes / 16;
    if (e == hipSuccess) {   // one untimed read, then the timed ones
        k_read_rate<<<grid, kBlock, 0, nullptr>>>((const float4 *)buf, n4, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    for (int32_t r = 0; e == hipSuccess && r < reps; ++r) {
        k_read_rate<<<grid, kBlock, 0, nullptr>>>((const float4 *)buf, n4, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return SISPH_E_DEVICE;
    *us = (double)ms * 1e3 / reps;
    return SISPH_OK;
}

extern "C" int32_t sisph_debug_gtvf_short(sisph_ctx *ctx, int32_t on, int32_t *used) {
    if (!ctx || on < -1 || on > 1) return SISPH_E_INVAL;
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    const bool can = make_params(&ctx->desc).g_sub != 0;   // its buffers exist
    if (on == 1 && !can) return fail(ctx, SISPH_E_INVAL, "this case has no GTVF short lists");
    if (on >= 0) {
        ctx->P.g_sub = on && can ? 1 : 0;
        ctx->T = single_target(ctx);
        drop_graphs(ctx->g_pre, ctx->g_post);   // captured with the old parameters
    }
    if (used) {
        Control C;
        HIPCHK(ctx, hipMemcpyAsync(&C, ctx->S.ctl, sizeof(Control), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        unsigned long long bound;
        std::memcpy(&bound, &ctx->P.g_D2, sizeof bound);
        *used = !ctx->P.g_sub ? 0 : (!C.g_full && C.g_disp_bits <= bound ? 1 : 2);
    }
    return SISPH_OK;
}

extern "C" int32_t sisph_persistent_fallbacks(sisph_ctx *ctx, int64_t *refused, int64_t *timed_out) {
    if (!ctx) return SISPH_E_INVAL;
    if (refused) *refused = ctx->persist_refused;
    if (timed_out) *timed_out = ctx->persist_timeouts;
    return SISPH_OK;
}

extern "C" int32_t sisph_persistent_info(sisph_ctx *ctx, int64_t *solves, int32_t *last) {
    if (!ctx) return SISPH_E_INVAL;
    if (solves) *solves = ctx->persist_solves;
    if (last) *last = ctx->persist_last ? 1 : 0;
    return SISPH_OK;
}

// ================================================================ batches
// Cases of one (dim, kernel, precision) share a device table and one launch
// per kernel; the per-kind maps give each workgroup its case.
struct Group {
    int32_t dim, kernel, precision;
    std::vector<sisph_ctx *> members;
    CaseEntry *d_tab = nullptr;
    int32_t *d_owner[K_COUNT] = {};
    int64_t *d_first[K_COUNT] = {};
    Control *d_ctl = nullptr;   // gathered control blocks [members]
    Control *h_ctl = nullptr;   // pinned mirror
    size_t owner_cap[K_COUNT] = {};   // entries of d_owner[k]
    size_t first_cap[K_COUNT] = {};   // entries of d_first[k]
    size_t case_cap = 0;              // entries of d_tab and d_ctl
    bool dirty = true;
    Target T{};
    hipGraphExec_t g_pre = nullptr, g_post = nullptr;   // fixed step segments (graph mode)
    int g_maxK = -1;
    // persistent batched solve of the wall-less Jacobi members: workgroup ->
    // case and the case's first workgroup over those members only, and the
    // launch's synchronisation words
    int32_t *d_powner = nullptr;
    int64_t *d_pfirst = nullptr;
    uint32_t *d_bsync = nullptr;
    size_t powner_cap = 0, bsync_cap = 0, case_cap_p = 0;
    int64_t ptotal = 0;               // workgroups of those members
    int32_t pcases = 0;               // how many members
    std::vector<int> pmembers;        // their indices in members
};

struct sisph_batch {
    int32_t max_cases;
    hipStream_t stream;
    bool use_graphs = false;
    hipStream_t cap_stream = nullptr;
    std::vector<sisph_ctx *> cases;   // attach order
    std::vector<Group> groups;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool use_persistent = true;       // batched persistent solves where they apply
    int64_t persist_launches = 0, persist_fallbacks = 0;
    std::string err;
};

static void free_group(Group &g) {
    drop_graphs(g.g_pre, g.g_post);
    if (g.d_tab) (void)hipFree(g.d_tab);
    for (int k = 0; k < K_COUNT; ++k) {
        if (g.d_owner[k]) (void)hipFree(g.d_owner[k]);
        if (g.d_first[k]) (void)hipFree(g.d_first[k]);
        g.d_owner[k] = nullptr;
        g.d_first[k] = nullptr;
        g.owner_cap[k] = 0;
        g.first_cap[k] = 0;
    }
    if (g.d_ctl) (void)hipFree(g.d_ctl);
    if (g.h_ctl) (void)hipHostFree(g.h_ctl);
    if (g.d_powner) (void)hipFree(g.d_powner);
    if (g.d_pfirst) (void)hipFree(g.d_pfirst);
    if (g.d_bsync) (void)hipFree(g.d_bsync);
    g.case_cap_p = 0;
    g.d_tab = nullptr;
    g.d_ctl = nullptr;
    g.h_ctl = nullptr;
    g.d_powner = nullptr;
    g.d_pfirst = nullptr;
    g.d_bsync = nullptr;
    g.powner_cap = g.bsync_cap = 0;
    g.case_cap = 0;
}

#define BCHK(b, expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (b)->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return SISPH_E_DEVICE;                                                      \
        }                                                                               \
    } while (0)

// Rebuilds a group's device table and workgroup maps after membership changed.
static int32_t rebuild_group(sisph_batch *b, Group &g) {
    drop_graphs(g.g_pre, g.g_post);   // captured against the old tables
    const size_t n = g.members.size();
    if (n > g.case_cap) {
        if (g.d_tab) (void)hipFree(g.d_tab);
        if (g.d_ctl) (void)hipFree(g.d_ctl);
        if (g.h_ctl) (void)hipHostFree(g.h_ctl);
        g.d_tab = nullptr;
        g.d_ctl = nullptr;
        g.h_ctl = nullptr;
        BCHK(b, hipMalloc((void **)&g.d_tab, sizeof(CaseEntry) * n));
        BCHK(b, hipMalloc((void **)&g.d_ctl, sizeof(Control) * n));
        BCHK(b, hipHostMalloc((void **)&g.h_ctl, sizeof(Control) * n, hipHostMallocDefault));
        g.case_cap = n;
    }
    std::vector<CaseEntry> tab(n);
    Target &T = g.T;
    T = Target{};
    T.batched = true;
    T.ncase = (int32_t)n;
    T.dim = g.dim;
    T.kernel = g.kernel;
    T.precision = g.precision;
    T.s = b->stream;
    for (auto *c : g.members) {
        T.adaptive |= c->P.adaptive_dt;
        T.packed |= c->P.packed;
        T.null_space |= c->P.null_space;
    }
    T.precheck = 1;
    for (int k = 0; k < K_COUNT; ++k) {
        std::vector<int32_t> owner;
        std::vector<int64_t> first(n);
        for (size_t c = 0; c < n; ++c) {
            const int64_t nb = kind_blocks(g.members[c]->P, k);
            tab[c].nblk[k] = nb;
            first[c] = (int64_t)owner.size();
            owner.insert(owner.end(), (size_t)nb, (int32_t)c);
        }
        T.total[k] = (int64_t)owner.size();
        // the two maps grow independently: the workgroup count can shrink
        // while the case count grows (large cases leave, small ones join)
        if (owner.size() > g.owner_cap[k] || !g.d_owner[k]) {
            if (g.d_owner[k]) (void)hipFree(g.d_owner[k]);
            g.d_owner[k] = nullptr;
            g.owner_cap[k] = 0;
            const size_t cap = std::max<size_t>(owner.size(), 1);
            BCHK(b, hipMalloc((void **)&g.d_owner[k], sizeof(int32_t) * cap));
            g.owner_cap[k] = cap;
        }
        if (n > g.first_cap[k] || !g.d_first[k]) {
            if (g.d_first[k]) (void)hipFree(g.d_first[k]);
            g.d_first[k] = nullptr;
            g.first_cap[k] = 0;
            const size_t cap = std::max<size_t>(n, 1);
            BCHK(b, hipMalloc((void **)&g.d_first[k], sizeof(int64_t) * cap));
            g.first_cap[k] = cap;
        }
        if (!owner.empty())
            BCHK(b, hipMemcpyAsync(g.d_owner[k], owner.data(), sizeof(int32_t) * owner.size(),
                                   hipMemcpyHostToDevice, b->stream));
        BCHK(b, hipMemcpyAsync(g.d_first[k], first.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, b->stream));
        T.owner[k] = g.d_owner[k];
        T.first[k] = g.d_first[k];
    }
    for (size_t c = 0; c < n; ++c) {
        tab[c].P = g.members[c]->P;
        tab[c].S = g.members[c]->S;
    }
    // the wall-less Jacobi members, for the persistent batched solve
    {
        std::vector<int32_t> powner;
        std::vector<int64_t> pfirst(n, -1);
        g.pmembers.clear();
        for (size_t c = 0; c < n; ++c) {
            const Params &P = g.members[c]->P;
            if (P.nw > 0 || P.solver != SISPH_JACOBI) continue;
            const int64_t nb = kind_blocks(P, K_FLUID);
            pfirst[c] = (int64_t)powner.size();
            powner.insert(powner.end(), (size_t)nb, (int32_t)c);
            g.pmembers.push_back((int)c);
        }
        g.ptotal = (int64_t)powner.size();
        g.pcases = (int32_t)g.pmembers.size();
        if (g.ptotal > 0) {
            if ((size_t)g.ptotal > g.powner_cap || !g.d_powner) {
                if (g.d_powner) (void)hipFree(g.d_powner);
                g.d_powner = nullptr;
                g.powner_cap = 0;
                BCHK(b, hipMalloc((void **)&g.d_powner, sizeof(int32_t) * (size_t)g.ptotal));
                g.powner_cap = (size_t)g.ptotal;
            }
            if (!g.d_pfirst || n > g.case_cap_p) {
                if (g.d_pfirst) (void)hipFree(g.d_pfirst);
                g.d_pfirst = nullptr;
                BCHK(b, hipMalloc((void **)&g.d_pfirst, sizeof(int64_t) * n));
                g.case_cap_p = n;
            }
            const size_t words = (size_t)batch_sync_words((int64_t)n);
            if (words > g.bsync_cap || !g.d_bsync) {
                if (g.d_bsync) (void)hipFree(g.d_bsync);
                g.d_bsync = nullptr;
                g.bsync_cap = 0;
                BCHK(b, hipMalloc((void **)&g.d_bsync, sizeof(uint32_t) * words));
                g.bsync_cap = words;
            }
            BCHK(b, hipMemcpyAsync(g.d_powner, powner.data(), sizeof(int32_t) * powner.size(), hipMemcpyHostToDevice,
                                   b->stream));
            BCHK(b, hipMemcpyAsync(g.d_pfirst, pfirst.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, b->stream));
        }
    }
    BCHK(b, hipMemcpyAsync(g.d_tab, tab.data(), sizeof(CaseEntry) * n, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    T.tab = g.d_tab;
    g.dirty = false;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_create(int32_t max_cases, void *hip_stream, sisph_batch **out) {
    if (!out || max_cases < 1) return SISPH_E_INVAL;
    sisph_batch *b = new sisph_batch();
    b->max_cases = max_cases;
    b->stream = (hipStream_t)hip_stream;
    if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess) {
        if (b->e0) (void)hipEventDestroy(b->e0);
        delete b;
        return SISPH_E_DEVICE;
    }
    *out = b;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_attach(sisph_batch *b, sisph_ctx *ctx) {
    if (!b || !ctx) return SISPH_E_INVAL;
    if (ctx->batch) return fail(ctx, SISPH_E_STATE, "context already attached to a batch");
    if (ctx->state != ST_READY) return fail(ctx, SISPH_E_STATE, "attach between steps only");
    if (ctx->stream != b->stream) return fail(ctx, SISPH_E_INVAL, "context and batch must share a stream");
    if (ctx->P.solver != SISPH_JACOBI) return fail(ctx, SISPH_E_INVAL, "BiCGStab contexts run alone");
    if ((int32_t)b->cases.size() >= b->max_cases) return fail(ctx, SISPH_E_NOMEM, "batch is full");
    Group *g = nullptr;
    for (auto &x : b->groups)
        if (x.dim == ctx->P.dim && x.kernel == ctx->P.kernel && x.precision == ctx->P.precision) g = &x;
    if (!g) {
        b->groups.emplace_back();
        g = &b->groups.back();
        g->dim = ctx->P.dim;
        g->kernel = ctx->P.kernel;
        g->precision = ctx->P.precision;
    }
    g->members.push_back(ctx);
    g->dirty = true;
    b->cases.push_back(ctx);
    ctx->batch = b;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_detach(sisph_batch *b, sisph_ctx *ctx) {
    if (!b || !ctx) return SISPH_E_INVAL;
    if (ctx->batch != b) return fail(ctx, SISPH_E_INVAL, "context is not attached to this batch");
    b->cases.erase(std::remove(b->cases.begin(), b->cases.end(), ctx), b->cases.end());
    for (auto &g : b->groups) {
        auto it = std::find(g.members.begin(), g.members.end(), ctx);
        if (it != g.members.end()) {
            g.members.erase(it);
            g.dirty = true;
        }
    }
    ctx->batch = nullptr;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_size(sisph_batch *b) { return b ? (int32_t)b->cases.size() : SISPH_E_INVAL; }

// One full step of one group; per-case results into the members' contexts.
static int32_t group_step(sisph_batch *b, Group &g) {
    if (g.members.empty()) return SISPH_OK;
    if (g.dirty) {
        int32_t st = rebuild_group(b, g);
        if (st != SISPH_OK) return st;
    }
    // the group's sweep variant is that of its largest case
    const sisph_ctx *largest = g.members[0];
    for (auto *c : g.members)
        if (c->P.nf > largest->P.nf) largest = c;
    g.T.variant = largest->variant;
    const Target &T = g.T;
    const size_t n = g.members.size();
    int64_t limit = 1, predicted = 1;
    int maxK = 0;
    for (auto *c : g.members) {
        const Params &P = c->P;
        limit = std::max<int64_t>(limit, (P.forced_iters > 0 ? P.forced_iters : P.max_iter) + 1);
        predicted = std::max<int64_t>(predicted, predict_iters(c));
        maxK = std::max(maxK, P.gtvf_K);
    }
    if (b->use_graphs) {
        if (!g.g_pre || g.g_maxK != maxK) {
            drop_graphs(g.g_pre, g.g_post);
            hipError_t e = capture_graph(b->cap_stream, T, seq_pre, &g.g_pre);
            if (e == hipSuccess)
                e = capture_graph(b->cap_stream, T, [maxK](const Target &t) { seq_post(t, maxK); }, &g.g_post);
            if (e != hipSuccess) {
                drop_graphs(g.g_pre, g.g_post);
                b->err = std::string("graph capture failed: ") + hipGetErrorString(e);
                return SISPH_E_DEVICE;
            }
            g.g_maxK = maxK;
        }
        BCHK(b, hipGraphLaunch(g.g_pre, b->stream));
    } else {
        seq_pre(T);
    }
    auto poll = [&](bool &done) -> int32_t {
        gather_control(T, g.d_ctl);
        BCHK(b, hipMemcpyAsync(g.h_ctl, g.d_ctl, sizeof(Control) * n, hipMemcpyDeviceToHost, b->stream));
        BCHK(b, hipStreamSynchronize(b->stream));
        done = true;
        for (size_t c = 0; c < n; ++c) done = done && g.h_ctl[c].done;
        return SISPH_OK;
    };
    // The wall-less Jacobi members first, in one persistent launch when
    // their workgroups can all be resident; the others (walls, BiCGStab)
    // then take per-launch sweeps, in which the finished cases return at once
    bool persistent_done = false;
    if (b->use_persistent && g.pcases > 0 && g.ptotal <= ppe_persistent_batch_capacity(T)) {
        // the starting iterates, kept in each case's binning scratch in case
        // the launch has to be redone with per-launch sweeps
        for (int c : g.pmembers) {
            const sisph_ctx *ctx = g.members[(size_t)c];
            BCHK(b, hipMemcpyAsync(ctx->S.tmp, ctx->S.p[0], sizeof(double) * (size_t)ctx->P.ntot,
                                   hipMemcpyDeviceToDevice, b->stream));
        }
        const int64_t words = batch_sync_words((int64_t)n);
        fill_u32(g.d_bsync, 0u, kBatchSyncStop, b->stream);
        fill_u32(g.d_bsync + kBatchSyncStop, 0xffffffffu, words - kBatchSyncStop, b->stream);
        uint32_t spins = kBarrierSpins;
        for (int c : g.pmembers) spins = std::min(spins, g.members[(size_t)c]->P.barrier_spins);
        const hipError_t e = ppe_persistent_batch(T, g.d_powner, g.d_pfirst, g.ptotal, g.d_bsync, g.pcases,
                                                  (int)limit, spins);
        if (e == hipSuccess) {
            uint32_t late = 0;
            BCHK(b, hipMemcpyAsync(&late, g.d_bsync, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream));
            BCHK(b, hipStreamSynchronize(b->stream));
            if (late) {
                // a workgroup never reached a barrier: the starting iterates
                // back, the solves set up again, per-launch sweeps for all
                b->persist_fallbacks += 1;
                for (int c : g.pmembers) {
                    const sisph_ctx *ctx = g.members[(size_t)c];
                    BCHK(b, hipMemcpyAsync(ctx->S.p[0], ctx->S.tmp, sizeof(double) * (size_t)ctx->P.ntot,
                                           hipMemcpyDeviceToDevice, b->stream));
                }
                seq_ppe_begin(T);
                BCHK(b, hipGetLastError());
            } else {
                b->persist_launches += 1;
                persistent_done = true;
            }
        } else {
            (void)hipGetLastError();   // refused: per-launch sweeps this step
            b->persist_fallbacks += 1;
        }
    }
    double sweep_ms = 0.0;
    int64_t launches = 0;
    if (!persistent_done || g.pcases < (int32_t)n) {
        int32_t st = ppe_loop(T, predicted, limit, b->e0, b->e1, sweep_ms, launches, poll, b->err);
        if (st != SISPH_OK) return st;
    }
    if (b->use_graphs) BCHK(b, hipGraphLaunch(g.g_post, b->stream));
    else seq_post(T, maxK);
    gather_control(T, g.d_ctl);
    BCHK(b, hipMemcpyAsync(g.h_ctl, g.d_ctl, sizeof(Control) * n, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    BCHK(b, hipGetLastError());
    for (size_t c = 0; c < n; ++c) {
        sisph_ctx *ctx = g.members[c];
        *ctx->h_ctl = g.h_ctl[c];
        record_iters(ctx, g.h_ctl[c].iter);
        ctx->sweep_effective += g.h_ctl[c].iter;
        ctx->nbr_stage = 1;
    }
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_step(sisph_batch *b, sisph_step_stats *per_case) {
    if (!b) return SISPH_E_INVAL;
    for (auto &g : b->groups) {
        int32_t st = group_step(b, g);
        if (st != SISPH_OK) return st;
    }
    // errors first (the most negative), else the largest warning
    int32_t err = SISPH_OK, warn = SISPH_OK;
    for (size_t c = 0; c < b->cases.size(); ++c) {
        sisph_ctx *ctx = b->cases[c];
        if (per_case) fill_stats(*ctx->h_ctl, ctx->P, per_case + c);
        std::string msg;
        const int32_t st = status_of(*ctx->h_ctl, ctx->P, &msg);
        if (st < 0) {
            ctx->err = msg;
            err = std::min(err, st);
        } else {
            warn = std::max(warn, st);
        }
    }
    return err < 0 ? err : warn;
}

extern "C" int32_t sisph_batch_set_graphs(sisph_batch *b, int32_t on) {
    if (!b) return SISPH_E_INVAL;
    b->use_graphs = on != 0;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_set_persistent(sisph_batch *b, int32_t on) {
    if (!b) return SISPH_E_INVAL;
    b->use_persistent = on != 0;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_persistent_info(sisph_batch *b, int64_t *launches, int64_t *fallbacks) {
    if (!b) return SISPH_E_INVAL;
    if (launches) *launches = b->persist_launches;
    if (fallbacks) *fallbacks = b->persist_fallbacks;
    return SISPH_OK;
}

extern "C" int32_t sisph_batch_destroy(sisph_batch *b) {
    if (!b) return SISPH_E_INVAL;
    (void)hipStreamSynchronize(b->stream);
    for (auto *c : b->cases) c->batch = nullptr;
    for (auto &g : b->groups) free_group(g);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    delete b;
    return SISPH_OK;
}

// ------------------------------------------------------------- autotune
extern "C" int32_t sisph_autotune(sisph_ctx *ctx, int32_t reps, int32_t *best, double *us) {
    if (!ctx || reps < 1) return SISPH_E_INVAL;
    if (attached(ctx)) return fail(ctx, SISPH_E_STATE, "context is attached to a batch");
    if (ctx->state != ST_READY || ctx->nbr_stage != 1)
        return fail(ctx, SISPH_E_STATE, "sisph_autotune needs one completed step");
    if (ctx->is_static) return fail(ctx, SISPH_E_STATE, "a context in the static workspace has no timing events");
    // launch 0 of a sweep reads the current pressure (iterate 0) and writes
    // only iterate 1, the FP32 copy and the partial sums: scratch between steps
    Target T = ctx->T;
    double t_us[kSweepVariants];
    int32_t win = 0;
    for (int v = 0; v < kSweepVariants; ++v) {
        T.variant = v;
        sweep_only(T, 0);   // warm-up
        HIPCHK(ctx, ev_record(ctx->evc[0], ctx->stream));
        for (int r = 0; r < reps; ++r) sweep_only(T, 0);
        HIPCHK(ctx, ev_record(ctx->evc[1], ctx->stream));
        HIPCHK(ctx, ev_sync(ctx->evc[1]));
        HIPCHK(ctx, hipGetLastError());
        float ms = 0.f;
        HIPCHK(ctx, ev_elapsed(&ms, ctx->evc[0], ctx->evc[1]));
        t_us[v] = ms * 1e3 / reps;
        if (us) us[v] = t_us[v];
        if (v == 0 || t_us[v] < t_us[win]) win = v;
    }
    ctx->variant = win;
    ctx->T.variant = win;
    if (best) *best = win;
    return SISPH_OK;
}

extern "C" int32_t sisph_set_variant(sisph_ctx *ctx, int32_t variant) {
    if (!ctx || variant < 0 || variant >= kSweepVariants) return SISPH_E_INVAL;
    ctx->variant = variant;
    ctx->T.variant = variant;
    return SISPH_OK;
}

extern "C" int32_t sisph_get_variant(sisph_ctx *ctx) { return ctx ? ctx->variant : SISPH_E_INVAL; }

extern "C" int32_t sisph_set_graphs(sisph_ctx *ctx, int32_t on) {
    if (!ctx) return SISPH_E_INVAL;
    if (on && ctx->is_static) return fail(ctx, SISPH_E_STATE, "a context in the static workspace captures no graphs");
    ctx->use_graphs = on != 0;
    return SISPH_OK;
}

extern "C" int32_t sisph_set_persistent(sisph_ctx *ctx, int32_t on) {
    if (!ctx) return SISPH_E_INVAL;
    ctx->use_persistent = on != 0;
    return SISPH_OK;
}

extern "C" int32_t sisph_destroy(sisph_ctx *ctx) {
    if (!ctx) return SISPH_E_INVAL;
    if (ctx->batch) (void)sisph_batch_detach(ctx->batch, ctx);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->is_static) {   // nothing of its own to free
        ctx->is_static = false;
        release_static(ctx);
        return SISPH_OK;
    }
    drop_graphs(ctx->g_pre, ctx->g_post);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->h_ctl) (void)hipHostFree(ctx->h_ctl);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->evc)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->kev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return SISPH_OK;
}

extern "C" const char *sisph_status_string(int32_t status) {
    switch (status) {
    case SISPH_OK: return "ok";
    case SISPH_WARN_MAXITER: return "PPE stopped at max_iter before reaching the tolerance";
    case SISPH_E_INVAL: return "invalid descriptor or argument";
    case SISPH_E_NOMEM: return "workspace or neighbour capacity too small";
    case SISPH_E_DEVICE: return "HIP runtime error";
    case SISPH_E_STATE: return "call out of order";
    case SISPH_E_NONFINITE: return "non-finite value in the PPE residual";
    default: return "unknown status";
    }
}

extern "C" const char *sisph_last_error(sisph_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return g_static_err_set ? g_static_err : g_create_err.c_str();
}
