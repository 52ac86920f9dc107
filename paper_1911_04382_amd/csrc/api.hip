// C ABI of the library (include/grass.h) and the host-side drivers: one
// embedding pass, the filtering step, and the iterative densification loop of
// Sec. IV-D of the paper.
#include <chrono>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "driver.h"
#include "embed.h"
#include "graph.h"
#include "kern.h"
#include "lsst.h"
#include "profiler.h"
#include "select.h"

namespace grass {
thread_local Profiler *g_prof = nullptr;
thread_local LaunchSched *g_sched = nullptr;
namespace {

// Everything one call needs, planned over one arena.
template <typename T>
struct Session {
    Dims d;
    Topo t;
    SetupTmp st;
    Vecs<T> v;
};

template <typename T>
void plan_session(Arena &a, long long n, long long m, int k, int prec, Session<T> &S) {
    S.d = make_dims(n, m, k, prec);
    plan_topo(a, S.d, S.t, S.st);
    plan_vecs<T>(a, S.d, S.v);
}

size_t plan_bytes(long long n, long long m, int k, int prec) {
    Arena a;
    a.dry = true;
    if (prec == 64) {
        Session<double> S;
        plan_session<double>(a, n, m, k, prec, S);
    } else {
        Session<float> S;
        plan_session<float>(a, n, m, k, prec, S);
    }
    return a.off + 256;
}

size_t plan_solve_bytes(long long n, long long m, int k, int prec) {
    Arena a;
    a.dry = true;
    if (prec == 64) {
        Session<double> S;
        plan_session<double>(a, n, m, k, prec, S);
        SddVecs<double> B;
        plan_sdd<double>(a, S.d, B);
    } else {
        Session<float> S;
        plan_session<float>(a, n, m, k, prec, S);
        SddVecs<float> B;
        plan_sdd<float>(a, S.d, B);
    }
    return a.off + 256;
}

size_t plan_partition_bytes(long long n, long long m, int prec) {
    Arena a;
    a.dry = true;
    if (prec == 64) {
        Session<double> S;
        plan_session<double>(a, n, m, 1, prec, S);
        SddVecs<double> B;
        plan_sdd<double>(a, S.d, B);
        PartVecs<double> P;
        plan_part<double>(a, S.d, P);
    } else {
        Session<float> S;
        plan_session<float>(a, n, m, 1, prec, S);
        SddVecs<float> B;
        plan_sdd<float>(a, S.d, B);
        PartVecs<float> P;
        plan_part<float>(a, S.d, P);
    }
    return a.off + 256;
}

void check_opts(const grass_opts &o) {
    require(o.k >= 1 && o.k <= kMaxK, GRASS_ERR_INVALID, "k must be in 1..64");
    require(o.t >= 1 && o.t <= 64, GRASS_ERR_INVALID, "t must be in 1..64");
    require(o.precision == 32 || o.precision == 64, GRASS_ERR_INVALID, "precision must be 32 or 64");
    require(o.sigma2 >= 1.0 && std::isfinite(o.sigma2), GRASS_ERR_INVALID, "sigma2 must be >= 1");
    require(o.max_iters >= 0, GRASS_ERR_INVALID, "max_iters must be >= 0");
    require(o.budget_frac >= 0.0, GRASS_ERR_INVALID, "budget_frac must be >= 0");
    require(o.lambda_steps >= 0 && o.lambda_steps <= 4096, GRASS_ERR_INVALID, "lambda_steps out of range");
}

// Bind the arena to the caller's workspace, or to the context's own memory.
Arena bind_arena(grass_ctx *ctx, void *ws, size_t ws_bytes, size_t need) {
    Arena a;
    if (ws) {
        require(ws_bytes >= need, GRASS_ERR_OOM,
                "workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(need) + " bytes");
        a.base = static_cast<char *>(ws);
        a.cap = ws_bytes;
    } else {
        if (ctx->own_bytes < need) {
            if (ctx->own_ws) GR_HIP(hipFree(ctx->own_ws));
            ctx->own_ws = nullptr;
            ctx->own_bytes = 0;
            if (hipMalloc(&ctx->own_ws, need) != hipSuccess) {
                (void)hipGetLastError();
                throw Error(GRASS_ERR_OOM, "device allocation of " + std::to_string(need) + " bytes failed");
            }
            ctx->own_bytes = need;
        }
        a.base = static_cast<char *>(ctx->own_ws);
        a.cap = ctx->own_bytes;
    }
    return a;
}

void check_device_flags(Topo &t, hipStream_t s) {
    unsigned f = (unsigned)read_i32(reinterpret_cast<const int *>(t.devflags), s);
    require(!(f & DEVERR_SPIN), GRASS_ERR_DEVICE, "a bounded device wait expired (tree-solve look-back)");
    require(!(f & DEVERR_NONFINITE), GRASS_ERR_NONFINITE,
            "a NaN or infinity appeared in the power vectors or heats (the working precision overflowed)");
}

std::string sci(double x) {
    char b[32];
    std::snprintf(b, sizeof(b), "%.3e", x);
    return b;
}

// An L_P solve that ended above its FP64 target (or with a non-finite residual)
bool solve_failed(double resid64, const grass_opts &o) {
    const double rtol = o.pcg_rtol > 0 ? o.pcg_rtol : 1e-6;
    return !(resid64 <= rtol);
}

// Setup shared by every entry point: validation, CSR, subgraph mask, tree layout.
template <typename T>
void setup(Session<T> &S, const grass_graph &g, const uint8_t *p_mask, bool need_tree, hipStream_t s) {
    Topo &t = S.t;
    t.src = g.src;
    t.dst = g.dst;
    t.w = g.w;
    validate_graph(t, s);
    build_csr<T>(t, S.v, S.st, s);
    if (p_mask) {
        GR_HIP(hipMemcpyAsync(t.mask, p_mask, t.m, hipMemcpyDeviceToDevice, s));
    } else {
        boruvka(t, S.st, t.mask, s);
    }
    if (need_tree) {
        build_tree<T>(t, S.v, S.d, S.st, s);
        build_pcsr<T>(t, S.v, s);
        S.d.p_nnz = read_i32(t.prow + t.n, s);
    }
    init_greedy_state(t, s);
    fill_u32(t.devflags, 4, 0u, s);
}

struct PassResult {
    PassScalars sc;
    long long pcg_iters = 0;
    double resid64 = 0.0;
};

// One pass of Sec. III-F: h0 (eq. 28), t steps of h <- L_P^+ L_G h (eq. 29), heat
// (eqs. 31, 35, 55) and the estimates (Sec. IV-C). Vectors are rescaled between
// steps by a power of two common to all of them (exact; heat ratios unchanged).
template <typename T>
PassResult run_pass(Session<T> &S, const grass_opts &o, int pass, bool use_pcg, T *heat, hipStream_t s) {
    Dims &d = S.d;
    Topo &t = S.t;
    Vecs<T> &v = S.v;
    PassResult pr;
    T *H = v.H, *Y = v.Y;
    if (use_pcg && !std::is_same<T, double>::value) {
        // passes that solve with L_P keep h0 and every right-hand side L_G h in FP64:
        // rounding a right-hand side to FP32 adds white noise whose smooth part, which
        // an ill-conditioned L_P amplifies, outweighs the right-hand side's own
        Vecs<double> vd;
        vd.part = v.part;
        vd.red = v.red;
        start_vectors<double>(d, o.seed, pass, v.x64, vd, s);
    } else {
        start_vectors<T>(d, o.seed, pass, H, v, s);
    }
    unsigned long long *absmax = v.u64s + U_ABSMAX;
    int steps = o.lambda_steps > o.t ? o.lambda_steps : o.t;
    for (int step = 1; step <= steps; step++) {
        // after an L_P solve its FP64 solution is at hand (H is it rounded to T): the
        // next product reads it and keeps the right-hand side in FP64
        const bool rhs64 = use_pcg && (step > 1 || !std::is_same<T, double>::value);
        if (rhs64)
            lap_apply_x64(t, d, v.x64, v.b64, step > 1 ? absmax : nullptr, v.eg.lrow, v.eg.nlong, s);
        else
            lap_apply<T>(d, t.rowptr, t.col, v.cval, v.eg, H, Y, -1, step > 1 ? absmax : nullptr, nullptr, s);
        fill_u32(reinterpret_cast<unsigned *>(absmax), 2, 0u, s);
        if (!use_pcg) {
            tree_solve<T>(t, v, d, Y, Y, nullptr, nullptr, absmax, s);
            std::swap(H, Y);
        } else {
            SolveInfo si = pcg_solve<T>(t, v, d, Y, H, o, s, rhs64 ? v.b64 : nullptr);
            pr.pcg_iters += si.iters;
            pr.resid64 = std::max(pr.resid64, si.resid64);
        }
        // after an L_P solve the FP64 solution is at hand: the scorer takes its
        // differences there (in FP32 runs H is that solution rounded to FP32)
        const double *h64 = use_pcg ? v.x64 : nullptr;
        if (step == o.t) {
            score_edges<T>(t, v, d, H, heat, s, h64);
            if (steps > o.t)
                GR_HIP(hipMemcpyAsync(v.u64s + 4, v.u64s + U_HMAX, 8, hipMemcpyDeviceToDevice, s));
        }
    }
    if (steps > o.t) {
        score_edges<T>(t, v, d, H, (T *)nullptr, s, use_pcg ? v.x64 : nullptr);  // Rayleigh quotient of the continued vectors
        GR_HIP(hipMemcpyAsync(v.u64s + U_HMAX, v.u64s + 4, 8, hipMemcpyDeviceToDevice, s));
    }
    pr.sc = finish_estimates<T>(t, v, d, s);
    check_device_flags(t, s);
    return pr;
}

double theta_of(double sigma2, double lmin, double lmax, int t) {
    // eq. (58): (sigma2 lambda_min / lambda_max)^(2t+1) by repeated multiplication
    double base = sigma2 * lmin / lmax;
    double r = base;
    for (int i = 0; i < 2 * t; i++) r *= base;
    return r;
}

template <typename T>
grass_status sparsify_impl(grass_ctx *ctx, const grass_graph &g, const grass_opts &o, void *ws, size_t ws_bytes,
                           grass_result *res, hipStream_t s) {
    size_t need = plan_bytes(g.n, g.m, o.k, o.precision);
    Arena a = bind_arena(ctx, ws, ws_bytes, need);
    Session<T> S;
    plan_session<T>(a, g.n, g.m, o.k, o.precision, S);
    setup<T>(S, g, o.init_mask, true, s);
    Topo &t = S.t;
    long long cnt[3];
    count_mask(t, t.mask, cnt, s);
    require(cnt[2] == 0, GRASS_ERR_INVALID, "init_mask values must be 0, 1 or 2");
    long long tree_edges = cnt[0], added = cnt[1];
    long long budget = 0;
    if (o.budget_frac > 0.0) budget = std::max<long long>(1, (long long)std::floor(o.budget_frac * (double)g.n));
    T *scores = static_cast<T *>(res->scores);
    bool filtered = false;
    long long scored = 0, pcg_total = 0;
    PassResult pr;
    int pass = 0;
    double kappa = 0;
    bool failed = false;
    for (;; pass++) {
        auto t0 = std::chrono::steady_clock::now();
        pr = run_pass<T>(S, o, pass, added > 0, S.v.heat, s);
        long long m_off = g.m - tree_edges - added;
        kappa = pr.sc.lambda_max / pr.sc.lambda_min;
        scored += m_off;
        pcg_total += pr.pcg_iters;
        bool stop = kappa <= o.sigma2 || m_off == 0 || pass >= o.max_iters;
        grass_pass_stats ps{};
        ps.pass = pass;
        ps.lambda_max = pr.sc.lambda_max;
        ps.lambda_min = pr.sc.lambda_min;
        ps.kappa = kappa;
        ps.heat_max = pr.sc.heat_max;
        ps.m_off = m_off;
        ps.pcg_iters = pr.pcg_iters;
        ps.pcg_resid64 = pr.resid64;
        if (added > 0 && solve_failed(pr.resid64, o)) {
            // heats from an inaccurate solve are not trusted: select nothing from them
            ps.flags |= GRASS_PASS_SOLVE_FAILED;
            failed = true;
            stop = true;
        }
        if (!stop) {
            ps.theta = theta_of(o.sigma2, pr.sc.lambda_min, pr.sc.lambda_max, o.t);
            SelectOut so;
            {
                ProfScope sc(PK_SELECT, 0.0, s);
                so = select_edges<T>(t, S.d, S.v.heat, ps.theta, pr.sc.heat_max, o.sim_hops, budget, scores, s);
            }
            ps.candidates = so.candidates;
            ps.accepted = so.accepted;
            filtered = true;
            added += so.accepted;
            build_pcsr<T>(t, S.v, s);
            S.d.p_nnz = read_i32(t.prow + t.n, s);
        } else if (!filtered && scores && !failed) {
            normalized_scores<T>(t, S.v.heat, pr.sc.heat_max, scores, s);
        }
        GR_HIP(hipStreamSynchronize(s));
        ps.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (res->trace && pass < res->trace_cap) res->trace[pass] = ps;
        if (stop) break;
    }
    if (res->edge_mask) GR_HIP(hipMemcpyAsync(res->edge_mask, t.mask, g.m, hipMemcpyDeviceToDevice, s));
    GR_HIP(hipStreamSynchronize(s));
    if (res->summary) {
        grass_summary &sm = *res->summary;
        sm.lambda_max = pr.sc.lambda_max;
        sm.lambda_min = pr.sc.lambda_min;
        sm.kappa = kappa;
        sm.pcg_resid64 = pr.resid64;
        sm.heat_max = pr.sc.heat_max;
        sm.passes = pass + 1;
        sm.tree_edges = tree_edges;
        sm.added_edges = added;
        sm.scored_edges = scored;
        sm.pcg_iters = pcg_total;
    }
    if (failed)
        throw Error(GRASS_ERR_SOLVE, "pass " + std::to_string(pass) + ": an L_P solve ended at FP64 relative residual " +
                                         sci(pr.resid64) + " > pcg_rtol " + sci(o.pcg_rtol) +
                                         "; edge_mask holds the subgraph before it");
    return kappa <= o.sigma2 ? GRASS_OK : GRASS_NOT_CONVERGED;
}

// Sec. V-E: L_G x = b with the subgraph of p_mask (or the spanning tree) as the
// preconditioner.
template <typename T>
grass_status solve_impl(grass_ctx *ctx, const grass_graph &g, const uint8_t *p_mask, const grass_opts &o,
                        const T *b, T *x, double rtol, int maxit, grass_solve_info *info, void *ws, size_t ws_bytes,
                        hipStream_t s) {
    size_t need = plan_solve_bytes(g.n, g.m, o.k, o.precision);
    Arena a = bind_arena(ctx, ws, ws_bytes, need);
    Session<T> S;
    plan_session<T>(a, g.n, g.m, o.k, o.precision, S);
    SddVecs<T> B;
    plan_sdd<T>(a, S.d, B);
    setup<T>(S, g, p_mask, true, s);
    long long cnt[3];
    count_mask(S.t, S.t.mask, cnt, s);
    require(cnt[2] == 0, GRASS_ERR_INVALID, "p_mask values must be 0, 1 or 2");
    auto t0 = std::chrono::steady_clock::now();
    SddInfo si = sdd_solve<T>(S.t, S.v, S.d, B, b, x, rtol, maxit, cnt[1] == 0, o, s);
    GR_HIP(hipStreamSynchronize(s));
    check_device_flags(S.t, s);
    if (info) {
        info->iters = si.iters;
        info->inner_iters = si.inner;
        info->resid = si.resid;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->added_edges = cnt[1];
    }
    return si.resid <= rtol ? GRASS_OK : GRASS_NOT_CONVERGED;
}

// Sec. V-F: the sign cut of an approximate Fiedler vector from inverse power steps
// through the sparsifier-preconditioned solver (one vector: k = 1).
template <typename T>
grass_status partition_impl(grass_ctx *ctx, const grass_graph &g, const uint8_t *p_mask, const grass_opts &o,
                            int steps, double rtol, T *u, uint8_t *side, grass_partition_info *info, void *ws,
                            size_t ws_bytes, hipStream_t s) {
    size_t need = plan_partition_bytes(g.n, g.m, o.precision);
    Arena a = bind_arena(ctx, ws, ws_bytes, need);
    Session<T> S;
    plan_session<T>(a, g.n, g.m, 1, o.precision, S);
    SddVecs<T> B;
    plan_sdd<T>(a, S.d, B);
    PartVecs<T> P;
    plan_part<T>(a, S.d, P);
    setup<T>(S, g, p_mask, true, s);
    long long cnt[3];
    count_mask(S.t, S.t.mask, cnt, s);
    require(cnt[2] == 0, GRASS_ERR_INVALID, "p_mask values must be 0, 1 or 2");
    grass_opts o1 = o;
    o1.k = 1;
    auto t0 = std::chrono::steady_clock::now();
    PartInfo pi = partition_run<T>(S.t, S.v, S.d, B, P, u, side, steps, rtol, o.pcg_max_iters > 0 ? o.pcg_max_iters : 1000,
                                   cnt[1] == 0, o1, s);
    GR_HIP(hipStreamSynchronize(s));
    check_device_flags(S.t, s);
    if (info) {
        info->steps = steps;
        info->outer_iters = pi.outer;
        info->inner_iters = pi.inner;
        info->resid = pi.resid;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return pi.resid <= rtol ? GRASS_OK : GRASS_NOT_CONVERGED;
}

template <typename T>
grass_status embed_impl(grass_ctx *ctx, const grass_graph &g, const uint8_t *p_mask, const grass_opts &o, int pass,
                        T *heat, grass_pass_stats *stats, void *ws, size_t ws_bytes, hipStream_t s) {
    size_t need = plan_bytes(g.n, g.m, o.k, o.precision);
    Arena a = bind_arena(ctx, ws, ws_bytes, need);
    Session<T> S;
    plan_session<T>(a, g.n, g.m, o.k, o.precision, S);
    require(p_mask != nullptr, GRASS_ERR_INVALID, "p_mask is required");
    setup<T>(S, g, p_mask, true, s);
    long long cnt[3];
    count_mask(S.t, S.t.mask, cnt, s);
    require(cnt[2] == 0, GRASS_ERR_INVALID, "p_mask values must be 0, 1 or 2");
    auto t0 = std::chrono::steady_clock::now();
    PassResult pr = run_pass<T>(S, o, pass, cnt[1] > 0, heat ? heat : S.v.heat, s);
    GR_HIP(hipStreamSynchronize(s));
    if (stats) {
        grass_pass_stats ps{};
        ps.pass = pass;
        ps.lambda_max = pr.sc.lambda_max;
        ps.lambda_min = pr.sc.lambda_min;
        ps.kappa = pr.sc.lambda_max / pr.sc.lambda_min;
        ps.heat_max = pr.sc.heat_max;
        ps.m_off = g.m - cnt[0] - cnt[1];
        ps.pcg_iters = pr.pcg_iters;
        ps.pcg_resid64 = pr.resid64;
        ps.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (cnt[1] > 0 && solve_failed(pr.resid64, o)) ps.flags |= GRASS_PASS_SOLVE_FAILED;
        *stats = ps;
    }
    if (cnt[1] > 0 && solve_failed(pr.resid64, o))
        throw Error(GRASS_ERR_SOLVE, "an L_P solve ended at FP64 relative residual " + sci(pr.resid64) +
                                         " > pcg_rtol " + sci(o.pcg_rtol));
    return GRASS_OK;
}

template <typename T>
grass_status select_impl(grass_ctx *ctx, const grass_graph &g, uint8_t *p_mask, const grass_opts &o, const T *heat,
                         double lmax, double lmin, grass_pass_stats *stats, T *scores, void *ws, size_t ws_bytes,
                         hipStream_t s) {
    size_t need = plan_bytes(g.n, g.m, o.k, o.precision);
    Arena a = bind_arena(ctx, ws, ws_bytes, need);
    Session<T> S;
    plan_session<T>(a, g.n, g.m, o.k, o.precision, S);
    require(p_mask != nullptr && heat != nullptr, GRASS_ERR_INVALID, "p_mask and heat are required");
    require(lmax > 0 && lmin > 0, GRASS_ERR_INVALID, "lambda estimates must be > 0");
    setup<T>(S, g, p_mask, false, s);
    double hmax = heat_max_off<T>(S.t, heat, s);  // over the edges not in P
    long long budget = 0;
    if (o.budget_frac > 0.0) budget = std::max<long long>(1, (long long)std::floor(o.budget_frac * (double)g.n));
    double th = theta_of(o.sigma2, lmin, lmax, o.t);
    SelectOut so = select_edges<T>(S.t, S.d, heat, th, hmax, o.sim_hops, budget, scores, s);
    GR_HIP(hipMemcpyAsync(p_mask, S.t.mask, g.m, hipMemcpyDeviceToDevice, s));
    GR_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->theta = th;
        stats->heat_max = hmax;
        stats->candidates = so.candidates;
        stats->accepted = so.accepted;
    }
    return GRASS_OK;
}

template <typename F>
grass_status guarded(grass_ctx *ctx, F f, bool profile = true) {
    if (!ctx) return GRASS_ERR_INVALID;
    struct Bind {
        Bind(Profiler *p) { g_prof = p; }
        ~Bind() {
            if (g_prof) g_prof->resolve();
            g_prof = nullptr;
        }
    };
    try {
        GR_HIP(hipSetDevice(ctx->device));
        Bind bind(profile ? &ctx->prof : nullptr);
        grass_status st = f();
        ctx->last_error.clear();
        return st;
    } catch (const Error &e) {
        ctx->last_error = e.what();
        return e.code;
    } catch (const std::exception &e) {
        ctx->last_error = e.what();
        return GRASS_ERR_DEVICE;
    }
}

void check_graph(const grass_graph *g) {
    require(g && g->src && g->dst && g->w, GRASS_ERR_INVALID, "graph pointers must be set");
    require(g->n >= 2 && g->m >= 1, GRASS_ERR_INVALID, "graph needs n >= 2 and m >= 1");
}

}  // namespace

void check_graph_args(const grass_graph *g) { check_graph(g); }
void check_opts_args(const grass_opts &o) { check_opts(o); }
size_t sparsify_bytes(const grass_graph &g, const grass_opts &o) { return plan_bytes(g.n, g.m, o.k, o.precision); }
grass_status sparsify_run(grass_ctx *ctx, const grass_graph &g, const grass_opts &o, void *ws, size_t ws_bytes,
                          grass_result *res, hipStream_t s) {
    require(ws != nullptr, GRASS_ERR_INVALID, "a workspace is required");
    if (o.precision == 64) return sparsify_impl<double>(ctx, g, o, ws, ws_bytes, res, s);
    return sparsify_impl<float>(ctx, g, o, ws, ws_bytes, res, s);
}

}  // namespace grass

using namespace grass;

// The workspace of grass_sparsify_static: a device array of fixed size, one copy per
// GPU, held until the process ends. Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in for the device symbol); it
// uses the device address that hipGetSymbolAddress returns for each GPU.
static __device__ __align__(256) unsigned char scratch[GRASS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each GPU

// Resolve `scratch` on `device` once (that device current); returns its address.
void *resolve_scratch(int device) {
    require(device >= 0 && device < kMaxDevices, GRASS_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        GR_HIP(hipGetDevice(&prev));
        GR_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            throw Error(GRASS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}
}  // namespace

extern "C" {

grass_status grass_create(int device, grass_ctx **out) {
    if (!out) return GRASS_ERR_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return GRASS_ERR_DEVICE;
    }
    void *sp = nullptr;
    try {
        sp = resolve_scratch(device);
    } catch (const Error &) {
        return GRASS_ERR_DEVICE;
    }
    *out = new grass_ctx();
    (*out)->device = device;
    (*out)->static_ws = sp;
    return GRASS_OK;
}

void grass_destroy(grass_ctx *ctx) {
    if (!ctx) return;
    if (ctx->own_ws) {
        (void)hipSetDevice(ctx->device);
        (void)hipFree(ctx->own_ws);
    }
    delete ctx;
}

const char *grass_last_error(const grass_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

grass_opts grass_opts_default(void) {
    grass_opts o{};
    o.sigma2 = 100.0;
    o.k = 16;
    o.t = 2;
    o.seed = 0;
    o.max_iters = 50;
    o.budget_frac = 0.01;
    o.sim_hops = 1;
    o.lambda_steps = 0;
    o.pcg_rtol = 1e-6;
    o.pcg_max_iters = 8000;
    o.pcg_inner_rtol = 1e-2;
    o.pcg_max_outer = 50;
    o.precision = 32;
    o.init_mask = nullptr;
    return o;
}

size_t grass_workspace_bytes(int64_t n, int64_t m, const grass_opts *opts) {
    grass_opts o = opts ? *opts : grass_opts_default();
    if (n < 2 || m < 1 || o.k < 1 || o.k > kMaxK) return 0;
    return plan_bytes(n, m, o.k, o.precision == 64 ? 64 : 32);
}

grass_status grass_sparsify(grass_ctx *ctx, const grass_graph *g, const grass_opts *opts, void *workspace,
                            size_t ws_bytes, grass_result *res, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(opts && res, GRASS_ERR_INVALID, "opts and result are required");
        check_opts(*opts);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (opts->precision == 64) return sparsify_impl<double>(ctx, *g, *opts, workspace, ws_bytes, res, s);
        return sparsify_impl<float>(ctx, *g, *opts, workspace, ws_bytes, res, s);
    });
}

grass_status grass_sparsify_static(grass_ctx *ctx, const grass_graph *g, const grass_opts *opts, grass_result *res,
                                   void *stream) {
    return guarded(
        ctx,
        [&]() -> grass_status {
            check_graph(g);
            require(opts && res, GRASS_ERR_INVALID, "opts and result are required");
            check_opts(*opts);
            const size_t need = plan_bytes(g->n, g->m, opts->k, opts->precision);
            require(need <= GRASS_STATIC_SCRATCH_BYTES, GRASS_ERR_OOM,
                    "the graph needs " + std::to_string(need) + " bytes of workspace, more than the " +
                        std::to_string((size_t)GRASS_STATIC_SCRATCH_BYTES) +
                        " of the static scratch: use grass_sparsify with a workspace");
            require(ctx->static_ws != nullptr, GRASS_ERR_DEVICE, "the static scratch was not resolved");
            hipStream_t s = static_cast<hipStream_t>(stream);
            // the same driver and kernels as grass_sparsify, over the static scratch
            if (opts->precision == 64)
                return sparsify_impl<double>(ctx, *g, *opts, ctx->static_ws, GRASS_STATIC_SCRATCH_BYTES, res, s);
            return sparsify_impl<float>(ctx, *g, *opts, ctx->static_ws, GRASS_STATIC_SCRATCH_BYTES, res, s);
        },
        /*profile=*/false);  // per-kernel event timing creates events: not on this path
}

grass_status grass_spanning_tree(grass_ctx *ctx, const grass_graph *g, uint8_t *tree_mask, void *workspace,
                                 size_t ws_bytes, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(tree_mask != nullptr, GRASS_ERR_INVALID, "tree_mask is required");
        hipStream_t s = static_cast<hipStream_t>(stream);
        grass_opts o = grass_opts_default();
        o.k = 1;
        size_t need = plan_bytes(g->n, g->m, 1, 32);
        Arena a = bind_arena(ctx, workspace, ws_bytes, need);
        Session<float> S;
        plan_session<float>(a, g->n, g->m, 1, 32, S);
        S.t.src = g->src;
        S.t.dst = g->dst;
        S.t.w = g->w;
        validate_graph(S.t, s);
        boruvka(S.t, S.st, tree_mask, s);
        GR_HIP(hipStreamSynchronize(s));
        return GRASS_OK;
    });
}

size_t grass_low_stretch_tree_workspace_bytes(int64_t n, int64_t m) {
    if (n < 0 || m < 0) return 0;
    return lsst_bytes(n, m);
}

grass_status grass_low_stretch_tree(grass_ctx *ctx, const grass_graph *g, uint64_t seed, int32_t class_bits,
                                    uint8_t *tree_mask, void *workspace, size_t ws_bytes, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(tree_mask != nullptr, GRASS_ERR_INVALID, "tree_mask is required");
        require(class_bits >= 1 && class_bits <= 64, GRASS_ERR_INVALID, "class_bits must be in 1..64");
        hipStream_t s = static_cast<hipStream_t>(stream);
        Arena a = bind_arena(ctx, workspace, ws_bytes, lsst_bytes(g->n, g->m));
        Topo t;
        t.n = g->n;
        t.m = g->m;
        t.src = g->src;
        t.dst = g->dst;
        t.w = g->w;
        t.devflags = a.take<unsigned>(4);
        validate_graph(t, s);
        low_stretch_tree(t, a, seed, class_bits, tree_mask, s);
        GR_HIP(hipStreamSynchronize(s));
        return GRASS_OK;
    });
}

grass_status grass_embed(grass_ctx *ctx, const grass_graph *g, const uint8_t *p_mask, const grass_opts *opts,
                         int32_t pass, void *heat, grass_pass_stats *stats, void *workspace, size_t ws_bytes,
                         void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(opts != nullptr, GRASS_ERR_INVALID, "opts are required");
        check_opts(*opts);
        require(pass >= 0, GRASS_ERR_INVALID, "pass must be >= 0");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (opts->precision == 64)
            return embed_impl<double>(ctx, *g, p_mask, *opts, pass, static_cast<double *>(heat), stats, workspace,
                                      ws_bytes, s);
        return embed_impl<float>(ctx, *g, p_mask, *opts, pass, static_cast<float *>(heat), stats, workspace, ws_bytes,
                                 s);
    });
}

size_t grass_solve_workspace_bytes(int64_t n, int64_t m, const grass_opts *opts) {
    grass_opts o = opts ? *opts : grass_opts_default();
    if (n < 2 || m < 1 || o.k < 1 || o.k > kMaxK || (o.precision != 32 && o.precision != 64)) return 0;
    return plan_solve_bytes(n, m, o.k, o.precision);
}

grass_status grass_solve(grass_ctx *ctx, const grass_graph *g, const uint8_t *p_mask, const grass_opts *opts,
                         const void *b, void *x, double rtol, int32_t max_iters, grass_solve_info *info,
                         void *workspace, size_t ws_bytes, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(opts != nullptr, GRASS_ERR_INVALID, "opts are required");
        check_opts(*opts);
        require(b != nullptr && x != nullptr && b != x, GRASS_ERR_INVALID, "b and x must be distinct device arrays");
        require(rtol > 0.0 && rtol < 1.0, GRASS_ERR_INVALID, "rtol must be in (0, 1)");
        require(max_iters >= 1, GRASS_ERR_INVALID, "max_iters must be >= 1");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (opts->precision == 64)
            return solve_impl<double>(ctx, *g, p_mask, *opts, static_cast<const double *>(b), static_cast<double *>(x),
                                      rtol, max_iters, info, workspace, ws_bytes, s);
        return solve_impl<float>(ctx, *g, p_mask, *opts, static_cast<const float *>(b), static_cast<float *>(x), rtol,
                                 max_iters, info, workspace, ws_bytes, s);
    });
}

size_t grass_partition_workspace_bytes(int64_t n, int64_t m, const grass_opts *opts) {
    grass_opts o = opts ? *opts : grass_opts_default();
    if (n < 2 || m < 1 || (o.precision != 32 && o.precision != 64)) return 0;
    return plan_partition_bytes(n, m, o.precision);
}

grass_status grass_partition(grass_ctx *ctx, const grass_graph *g, const uint8_t *p_mask, const grass_opts *opts,
                             int32_t steps, double rtol, void *fiedler, uint8_t *side, grass_partition_info *info,
                             void *workspace, size_t ws_bytes, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(opts != nullptr, GRASS_ERR_INVALID, "opts are required");
        grass_opts o = *opts;
        o.k = 1;
        check_opts(o);
        require(fiedler != nullptr && side != nullptr, GRASS_ERR_INVALID, "fiedler and side are required");
        require(steps >= 1 && steps <= 1000, GRASS_ERR_INVALID, "steps must be in 1..1000");
        require(rtol > 0.0 && rtol < 1.0, GRASS_ERR_INVALID, "rtol must be in (0, 1)");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (o.precision == 64)
            return partition_impl<double>(ctx, *g, p_mask, o, steps, rtol, static_cast<double *>(fiedler), side, info,
                                          workspace, ws_bytes, s);
        return partition_impl<float>(ctx, *g, p_mask, o, steps, rtol, static_cast<float *>(fiedler), side, info,
                                     workspace, ws_bytes, s);
    });
}

grass_status grass_select(grass_ctx *ctx, const grass_graph *g, uint8_t *p_mask, const grass_opts *opts,
                          const void *heat, double lambda_max, double lambda_min, grass_pass_stats *stats,
                          void *scores, void *workspace, size_t ws_bytes, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        check_graph(g);
        require(opts != nullptr, GRASS_ERR_INVALID, "opts are required");
        check_opts(*opts);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (opts->precision == 64)
            return select_impl<double>(ctx, *g, p_mask, *opts, static_cast<const double *>(heat), lambda_max,
                                       lambda_min, stats, static_cast<double *>(scores), workspace, ws_bytes, s);
        return select_impl<float>(ctx, *g, p_mask, *opts, static_cast<const float *>(heat), lambda_max, lambda_min,
                                  stats, static_cast<float *>(scores), workspace, ws_bytes, s);
    });
}

grass_status grass_start_vectors(grass_ctx *ctx, int64_t n, int32_t k, uint64_t seed, int32_t pass,
                                 int32_t precision, void *out, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        require(n >= 1 && k >= 1 && k <= kMaxK && out, GRASS_ERR_INVALID, "bad start-vector arguments");
        require(precision == 32 || precision == 64, GRASS_ERR_INVALID, "precision must be 32 or 64");
        hipStream_t s = static_cast<hipStream_t>(stream);
        Dims d = make_dims(n, 1, k, precision);
        // only the reduction scratch is needed
        size_t need = (size_t)(2048 * kMaxK + RED_SLOTS * kMaxK + 64) * sizeof(double) + 1024;
        Arena a = bind_arena(ctx, nullptr, 0, need);
        if (precision == 64) {
            Vecs<double> v;
            v.part = a.take<double>(2048 * kMaxK + 64);
            v.red = a.take<double>(RED_SLOTS * kMaxK);
            start_vectors<double>(d, seed, pass, static_cast<double *>(out), v, s);
        } else {
            Vecs<float> v;
            v.part = a.take<double>(2048 * kMaxK + 64);
            v.red = a.take<double>(RED_SLOTS * kMaxK);
            start_vectors<float>(d, seed, pass, static_cast<float *>(out), v, s);
        }
        GR_HIP(hipStreamSynchronize(s));
        return GRASS_OK;
    });
}

grass_status grass_gram(grass_ctx *ctx, int64_t n, int32_t k, int32_t precision, const void *a, const void *b,
                        double *out, void *stream) {
    return guarded(ctx, [&]() -> grass_status {
        require(n >= 1 && k >= 1 && k <= kMaxK && a && b && out, GRASS_ERR_INVALID, "bad Gram arguments");
        require(precision == 32 || precision == 64, GRASS_ERR_INVALID, "precision must be 32 or 64");
        hipStream_t s = static_cast<hipStream_t>(stream);
        Dims d = make_dims(n, 1, k, precision);
        size_t need = (size_t)bpcg_part_doubles(d) * sizeof(double) + (size_t)bpcg_counters(d) * sizeof(int) + 1024;
        Arena ar = bind_arena(ctx, nullptr, 0, need);
        double *part = ar.take<double>((size_t)bpcg_part_doubles(d));
        int *cnt = ar.take<int>((size_t)bpcg_counters(d));
        if (precision == 64)
            block_gram<double>(d, static_cast<const double *>(a), static_cast<const double *>(b), part, cnt, out, s);
        else
            block_gram<float>(d, static_cast<const float *>(a), static_cast<const float *>(b), part, cnt, out, s);
        GR_HIP(hipStreamSynchronize(s));
        return GRASS_OK;
    });
}

grass_status grass_set_launch_mode(grass_ctx *ctx, int32_t mode, int32_t chunks_per_read) {
    if (!ctx) return GRASS_ERR_INVALID;
    if ((mode != GRASS_LAUNCH_KERNELS && mode != GRASS_LAUNCH_CAPTURED) || chunks_per_read < 0 ||
        chunks_per_read > 64) {
        ctx->last_error = "launch mode must be GRASS_LAUNCH_KERNELS or GRASS_LAUNCH_CAPTURED, chunks_per_read in 0..64";
        return GRASS_ERR_INVALID;
    }
    ctx->launch_mode = mode;
    ctx->launch_chunks = chunks_per_read;
    return GRASS_OK;
}

grass_status grass_launch_stats_read(grass_ctx *ctx, grass_launch_stats *out, int32_t reset) {
    if (!ctx || !out) return GRASS_ERR_INVALID;
    out->iterations = ctx->lstats.iterations.load();
    out->host_reads = ctx->lstats.host_reads.load();
    out->graph_replays = ctx->lstats.replays.load();
    out->captures = ctx->lstats.captures.load();
    if (reset) {
        ctx->lstats.iterations = 0;
        ctx->lstats.host_reads = 0;
        ctx->lstats.replays = 0;
        ctx->lstats.captures = 0;
    }
    return GRASS_OK;
}

grass_status grass_profile_enable(grass_ctx *ctx, uint32_t kinds) {
    if (!ctx) return GRASS_ERR_INVALID;
    ctx->prof.on = kinds != 0;
    ctx->prof.mask = kinds;
    ctx->prof.reset();
    return GRASS_OK;
}

int32_t grass_profile_read(const grass_ctx *ctx, grass_kernel_stats *out, int32_t cap) {
    static const char *names[PK_COUNT] = {"spmm_LG",  "spmm_LP",   "tree_up", "tree_down", "score",
                                          "gram_PQR", "r_update",  "gram_QZ", "p_update",  "p_normalize", "pcg_small",
                                          "resid64",  "start_vectors", "select", "spmm_LG64"};
    if (!ctx) return 0;
    int32_t n = 0;
    for (int i = 0; i < PK_COUNT && n < cap; i++) {
        if (!out) break;
        out[n].name = names[i];
        out[n].launches = ctx->prof.launches[i];
        out[n].total_ms = ctx->prof.ms[i];
        out[n].alg_bytes = ctx->prof.bytes[i];
        n++;
    }
    return out ? n : PK_COUNT;
}

}  // extern "C"
