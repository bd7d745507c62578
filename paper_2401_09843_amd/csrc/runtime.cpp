// Host runtime behind the C ABI of include/ns.h: contexts, sample groups,
// workspaces, twiddle and damping tables, the pass sequence of one
// right-hand-side evaluation, SSP-RK3 stages and hipGraph replay.
#include "../../include/ns.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "args.hpp"
#include "misc_kernels.hpp"

using namespace ns;

namespace ns {
#define NS_SIZES(X) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(60) X(64) X(80) X(96) X(120) X(128) X(256) X(512) X(1024)
#define NS_DECL(n) const SizeKernels* kernels_##n(bool f64);
NS_SIZES(NS_DECL)
#undef NS_DECL

const SizeKernels* find_kernels(int N, bool f64)
{
    switch (N) {
#define NS_CASE(n) \
    case n: return kernels_##n(f64);
        NS_SIZES(NS_CASE)
#undef NS_CASE
        default: return nullptr;
    }
}

int supported_sizes(int* out, int cap)
{
    static const int all[] = {
#define NS_LIST(n) n,
        NS_SIZES(NS_LIST)
#undef NS_LIST
    };
    const int cnt = (int)(sizeof(all) / sizeof(all[0]));
    for (int i = 0; i < cnt && i < cap; ++i) out[i] = all[i];
    return cnt;
}
}  // namespace ns

namespace {

thread_local std::string g_init_error;

// One group: every sample of the context with the same N, stored
// back-to-back so that each pass is a single launch for the whole group.
struct Group {
    int N = 0, K = 0, M = 0, Mx = 0, B = 0;
    std::vector<int> samples;  // context sample index of batch slot b
    const SizeKernels* kern = nullptr;
    long long MMx = 0;         // M * Mx, columns of a compact plane
    long long st = 0;          // compact state elements per sample, 3 M M Mx
    double eps = 0, m_cut = 0;
    void *U0 = nullptr, *U1 = nullptr;  // compact states
    void *A = nullptr, *Bw = nullptr, *C = nullptr;  // pass workspaces
    void *tw = nullptr, *rate = nullptr;
    double *dt = nullptr, *ones = nullptr;
};

}  // namespace

struct ns_ctx {
    ns_params prm{};
    std::vector<int> n;
    std::vector<int> group_of, slot_of;
    bool f64 = false;
    size_t rsz = 4;  // bytes per real
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<Group> groups;
    std::vector<void*> allocs;
    size_t bytes = 0;
    std::string err;
    bool failed = false;
    hipGraphExec_t step_exec = nullptr;
    hipGraph_t step_graph = nullptr;
    double* edev = nullptr;  // energy check scratch
    // pass profiler: events bracketing each launch while enabled
    bool profile = false;
    struct Rec {
        int pass;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

ns_status fail(ns_ctx* c, ns_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (st == NS_ERR_HIP) c->failed = true;
    } else {
        g_init_error = buf;
    }
    return st;
}

#define HIP_TRY(ctx, expr)                                                                                  \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) return fail((ctx), NS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define CHECK_STATE(ctx)                                                                          \
    do {                                                                                          \
        if (!(ctx)) return NS_ERR_ARG;                                                            \
        if ((ctx)->failed) return fail((ctx), NS_ERR_STATE, "context failed earlier: %s", (ctx)->err.c_str()); \
    } while (0)

ns_status dalloc(ns_ctx* c, void** p, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, NS_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    c->bytes += bytes;
    return NS_OK;
}

// tw[e] = exp(-2 pi i e / N), from long double, rounded to the working precision
template <typename R>
std::vector<R> twiddle_table(int N)
{
    std::vector<R> t(2 * (size_t)N);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int e = 0; e < N; ++e) {
        const long double a = 2.0L * pi * (long double)e / (long double)N;
        t[2 * e] = (R)cosl(a);
        t[2 * e + 1] = (R)(-sinl(a));
    }
    return t;
}

// damping rate eps |k|^{2s} Q(|k|) for |k|^2 = 0..3K^2 (eqs. (2.1)-(2.3))
template <typename R>
std::vector<R> rate_table(int K, double eps, double s, double m, int q_kind, double theta)
{
    std::vector<R> t(3 * (size_t)K * K + 1);
    for (size_t k2 = 0; k2 < t.size(); ++k2) {
        const double kabs = std::sqrt((double)k2);
        double q;
        if (kabs <= m) q = 0.0;
        else if (q_kind == 0) q = 1.0;
        else q = 1.0 - std::pow(m / kabs, (2.0 * s - 1.0) / theta);
        t[k2] = (R)(eps * std::pow((double)k2, s) * q);
    }
    return t;
}

ns_status upload(ns_ctx* c, void* dst, const void* src, size_t bytes)
{
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NS_OK;
}

ns_status setup_group(ns_ctx* c, Group& g)
{
    const int N = g.N;
    g.K = (N - 1) / 3;
    g.M = 2 * g.K + 1;
    g.Mx = g.K + 1;
    g.MMx = (long long)g.M * g.Mx;
    g.st = 3LL * g.M * g.MMx;
    g.B = (int)g.samples.size();
    g.kern = find_kernels(N, c->f64);
    if (!g.kern) return fail(c, NS_ERR_UNSUPPORTED, "grid size N=%d is not supported", N);
    const double s = c->prm.s;
    g.eps = c->prm.eps >= 0 ? c->prm.eps : 1e-3 * std::pow(32.0 / N, 2.0 * s - 1.0);
    g.m_cut = c->prm.m_cut >= 0 ? c->prm.m_cut : N / 3.0;
    const size_t cw = 2 * c->rsz;
    const long long B = g.B;
    ns_status st;
    if ((st = dalloc(c, &g.U0, cw * g.st * B))) return st;
    if ((st = dalloc(c, &g.U1, cw * g.st * B))) return st;
    if ((st = dalloc(c, &g.A, cw * 6ULL * N * g.MMx * B))) return st;
    if ((st = dalloc(c, &g.Bw, cw * 3ULL * N * N * g.Mx * B))) return st;
    if ((st = dalloc(c, &g.C, cw * 6ULL * N * N * g.Mx * B))) return st;
    if ((st = dalloc(c, &g.tw, cw * N))) return st;
    if ((st = dalloc(c, &g.rate, c->rsz * (3ULL * g.K * g.K + 1)))) return st;
    if ((st = dalloc(c, (void**)&g.dt, sizeof(double) * B))) return st;
    if ((st = dalloc(c, (void**)&g.ones, sizeof(double) * B))) return st;
    if (c->f64) {
        auto tw = twiddle_table<double>(N);
        auto rt = rate_table<double>(g.K, g.eps, s, g.m_cut, c->prm.q_kind, c->prm.theta);
        if ((st = upload(c, g.tw, tw.data(), tw.size() * sizeof(double)))) return st;
        if ((st = upload(c, g.rate, rt.data(), rt.size() * sizeof(double)))) return st;
    } else {
        auto tw = twiddle_table<float>(N);
        auto rt = rate_table<float>(g.K, g.eps, s, g.m_cut, c->prm.q_kind, c->prm.theta);
        if ((st = upload(c, g.tw, tw.data(), tw.size() * sizeof(float)))) return st;
        if ((st = upload(c, g.rate, rt.data(), rt.size() * sizeof(float)))) return st;
    }
    std::vector<double> ones(B, 1.0);
    if ((st = upload(c, g.ones, ones.data(), sizeof(double) * B))) return st;
    return NS_OK;
}

inline size_t cwb(const ns_ctx* c) { return 2 * c->rsz; }

hipEvent_t pool_event(ns_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// launch one pass, bracketed by events when the profiler is on
template <class F>
ns_status timed(ns_ctx* c, int pass, F&& launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->profile) {
        a = pool_event(c);
        b = pool_event(c);
        if (!a || !b) return fail(c, NS_ERR_HIP, "hipEventCreate failed");
        HIP_TRY(c, hipEventRecord(a, c->stream));
    }
    HIP_TRY(c, launch());
    if (c->profile) {
        HIP_TRY(c, hipEventRecord(b, c->stream));
        c->recs.push_back({pass, a, b});
    }
    return NS_OK;
}

// One right-hand-side evaluation for every sample of a group, reading the
// compact stage state us (and u0), writing out = ca u0 + cb us + cc dt F(us).
ns_status run_rhs(ns_ctx* c, Group& g, const void* us, void* out, const void* u0, double ca, double cb, double cc,
                  const double* dt)
{
    const SizeKernels* k = g.kern;
    const long long N = g.N, B = g.B, M = g.M, Mx = g.Mx, MMx = g.MMx;
    hipStream_t s = c->stream;
    // I1: [B][3][M][MMx] -> [B][3][N][MMx]
    ns_status st;
    ColArgs a1{us, g.A, g.tw, B * 3 * MMx, MMx, M * MMx, N * MMx, g.K, g.M, 1.0};
    if ((st = timed(c, 0, [&] { return k->col_inv(a1, s); }))) return st;
    // I2: [B*3*N][M][Mx] -> [B*3*N][N][Mx]
    ColArgs a2{g.A, g.Bw, g.tw, B * 3 * N * Mx, Mx, M * Mx, N * Mx, g.K, g.M, 1.0};
    if ((st = timed(c, 1, [&] { return k->col_inv(a2, s); }))) return st;
    // X: [B][3][N*N][Mx] -> [B][6][N*N][Mx]
    XArgs ax{g.Bw, g.C, g.tw, B * N * N / 2, N * N * Mx, N * N * Mx, 3 * N * N * Mx, 6 * N * N * Mx, g.K, 1.0 / N};
    if ((st = timed(c, 2, [&] { return k->x_rhs(ax, s); }))) return st;
    // F2: [B*6*N][N][Mx] -> [B*6*N][M][Mx]
    ColArgs a3{g.C, g.A, g.tw, B * 6 * N * Mx, Mx, N * Mx, M * Mx, g.K, g.M, 1.0 / N};
    if ((st = timed(c, 3, [&] { return k->col_fwd(a3, s); }))) return st;
    // F3: [B][6][N][MMx] -> compact [B][3][M][MMx]
    F3Args f{g.A, u0, us, out, g.tw, g.rate, dt, B * MMx, (int)MMx, g.Mx, g.K, g.M,
             6 * N * MMx, N * MMx, g.st, M * MMx, ca, cb, cc, 1.0 / N};
    if ((st = timed(c, 4, [&] { return k->f3_rhs(f, s); }))) return st;
    return NS_OK;
}

// One SSP-RK3 step (eq. (2.6)) of a group in place on U0, stages in U1.
ns_status rk3_step(ns_ctx* c, Group& g)
{
    ns_status st;
    // u1 = u + dt F(u)
    if ((st = run_rhs(c, g, g.U0, g.U1, nullptr, 0.0, 1.0, 1.0, g.dt))) return st;
    // u2 = 3/4 u + 1/4 u1 + 1/4 dt F(u1)
    if ((st = run_rhs(c, g, g.U1, g.U1, g.U0, 0.75, 0.25, 0.25, g.dt))) return st;
    // u^{n+1} = 1/3 u + 2/3 u2 + 2/3 dt F(u2)
    if ((st = run_rhs(c, g, g.U1, g.U0, g.U0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, g.dt))) return st;
    return NS_OK;
}

ns_status step_all(ns_ctx* c)
{
    ns_status st;
    for (Group& g : c->groups)
        if ((st = rk3_step(c, g))) return st;
    return NS_OK;
}

ns_status pack_all(ns_ctx* c, const void* const* uh, bool to_u0)
{
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        char* dst = (char*)(to_u0 ? g.U0 : g.U1) + cwb(c) * g.st * c->slot_of[i];
        HIP_TRY(c, launch_pack(c->f64, uh[i], dst, g.N, g.K, c->stream));
    }
    return NS_OK;
}

ns_status unpack_all(ns_ctx* c, void* const* uh, bool from_u0)
{
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        const char* src = (const char*)(from_u0 ? g.U0 : g.U1) + cwb(c) * g.st * c->slot_of[i];
        HIP_TRY(c, launch_unpack(c->f64, src, uh[i], g.N, g.K, c->stream));
    }
    return NS_OK;
}

ns_status check_ptrs(ns_ctx* c, const void* const* p, const char* what)
{
    if (!p) return fail(c, NS_ERR_ARG, "%s: null pointer array", what);
    for (size_t i = 0; i < c->n.size(); ++i)
        if (!p[i]) return fail(c, NS_ERR_ARG, "%s[%zu] is null", what, i);
    return NS_OK;
}

ns_status check_dt(ns_ctx* c, const double* dt)
{
    if (!dt) return fail(c, NS_ERR_ARG, "dt: null pointer");
    for (size_t i = 0; i < c->n.size(); ++i)
        if (!(std::isfinite(dt[i]) && dt[i] > 0)) return fail(c, NS_ERR_ARG, "dt[%zu] = %g must be finite and > 0", i, dt[i]);
    return NS_OK;
}

ns_status set_dt(ns_ctx* c, const double* dt)
{
    for (Group& g : c->groups) {
        std::vector<double> v(g.B);
        for (int b = 0; b < g.B; ++b) v[b] = dt[g.samples[b]];
        HIP_TRY(c, hipMemcpyAsync(g.dt, v.data(), sizeof(double) * g.B, hipMemcpyHostToDevice, c->stream));
        // the host vector dies here: wait for the copy
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return NS_OK;
}

ns_status ensure_graph(ns_ctx* c)
{
    if (c->step_exec) return NS_OK;
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->stream = user;
        return fail(c, NS_ERR_HIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    }
    ns_status st = step_all(c);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &graph);
    c->stream = user;
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(c, NS_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    c->step_graph = graph;
    HIP_TRY(c, hipGraphInstantiate(&c->step_exec, graph, nullptr, nullptr, 0));
    return NS_OK;
}

}  // namespace

extern "C" {

ns_status ns_supported_sizes(int32_t* sizes, int32_t cap, int32_t* count)
{
    if (!count || (cap > 0 && !sizes)) return NS_ERR_ARG;
    std::vector<int> tmp(64);
    int n = supported_sizes(tmp.data(), (int)tmp.size());
    for (int i = 0; i < n && i < cap; ++i) sizes[i] = tmp[i];
    *count = n;
    return NS_OK;
}

ns_status ns_init(const ns_params* p, void* hip_stream, ns_ctx** out)
{
    if (!out) return fail(nullptr, NS_ERR_ARG, "out is null");
    *out = nullptr;
    if (!p) return fail(nullptr, NS_ERR_ARG, "params is null");
    if (p->dtype != NS_F32 && p->dtype != NS_F64) return fail(nullptr, NS_ERR_ARG, "bad dtype %d", (int)p->dtype);
    if (p->nsamples < 1 || !p->n) return fail(nullptr, NS_ERR_ARG, "nsamples must be >= 1 with a size array");
    if (!(p->s >= 0) || !std::isfinite(p->s)) return fail(nullptr, NS_ERR_ARG, "s must be finite and >= 0");
    if (p->q_kind != 0 && p->q_kind != 1) return fail(nullptr, NS_ERR_ARG, "q_kind must be 0 or 1");
    if (p->q_kind == 1 && !(p->theta > 0)) return fail(nullptr, NS_ERR_ARG, "theta must be > 0 for q_kind 1");
    if (!std::isfinite(p->eps) || !std::isfinite(p->m_cut)) return fail(nullptr, NS_ERR_ARG, "eps and m_cut must be finite");
    for (int i = 0; i < p->nsamples; ++i) {
        if (!find_kernels(p->n[i], p->dtype == NS_F64))
            return fail(nullptr, NS_ERR_UNSUPPORTED, "grid size n[%d]=%d is not supported", i, p->n[i]);
    }
    ns_ctx* c = new ns_ctx;
    c->prm = *p;
    c->prm.n = nullptr;
    c->prm.tune_cache = nullptr;
    c->f64 = p->dtype == NS_F64;
    c->rsz = c->f64 ? 8 : 4;
    c->stream = (hipStream_t)hip_stream;
    c->n.assign(p->n, p->n + p->nsamples);
    c->group_of.resize(c->n.size());
    c->slot_of.resize(c->n.size());
    for (size_t i = 0; i < c->n.size(); ++i) {
        int gi = -1;
        for (size_t j = 0; j < c->groups.size(); ++j)
            if (c->groups[j].N == c->n[i]) gi = (int)j;
        if (gi < 0) {
            c->groups.emplace_back();
            c->groups.back().N = c->n[i];
            gi = (int)c->groups.size() - 1;
        }
        c->group_of[i] = gi;
        c->slot_of[i] = (int)c->groups[gi].samples.size();
        c->groups[gi].samples.push_back((int)i);
    }
    ns_status st = NS_OK;
    for (Group& g : c->groups)
        if ((st = setup_group(c, g))) break;
    if (st == NS_OK) st = dalloc(c, (void**)&c->edev, sizeof(double) * 4096);
    if (st != NS_OK) {
        g_init_error = c->err;
        ns_destroy(c);
        return st;
    }
    *out = c;
    return NS_OK;
}

ns_status ns_destroy(ns_ctx* c)
{
    if (!c) return NS_OK;
    (void)hipStreamSynchronize(c->stream);
    for (auto& r : c->recs) {
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
    if (c->step_graph) (void)hipGraphDestroy(c->step_graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
    return NS_OK;
}

const char* ns_last_error(const ns_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

ns_status ns_workspace_bytes(const ns_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return NS_ERR_ARG;
    *bytes = c->bytes;
    return NS_OK;
}

ns_status ns_sync(ns_ctx* c)
{
    CHECK_STATE(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NS_OK;
}

ns_status ns_profile(ns_ctx* c, int32_t enable)
{
    CHECK_STATE(c);
    c->profile = enable != 0;
    return NS_OK;
}

ns_status ns_profile_read(ns_ctx* c, double* ms, int64_t* count)
{
    CHECK_STATE(c);
    if (!ms || !count) return fail(c, NS_ERR_ARG, "ms and count must be non-null");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int p = 0; p < NS_NPASS; ++p) {
        ms[p] = 0.0;
        count[p] = 0;
    }
    for (auto& r : c->recs) {
        float t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&t, r.a, r.b));
        ms[r.pass] += t;
        count[r.pass] += 1;
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    return NS_OK;
}

ns_status ns_project(ns_ctx* c, void* const* uh)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat"))) return st;
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        HIP_TRY(c, launch_project(c->f64, uh[i], g.N, g.K, c->stream));
    }
    return NS_OK;
}

ns_status ns_forward(ns_ctx* c, const void* const* u, void* const* uh)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, u, "u_phys")) || (st = check_ptrs(c, (const void* const*)uh, "uhat"))) return st;
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        const long long N = g.N, M = g.M, Mx = g.Mx, MMx = g.MMx;
        hipStream_t s = c->stream;
        // x: real [3][N*N][N] -> [3][N*N][Mx]
        XArgs ax{u[i], g.C, g.tw, N * N / 2, N * N * N, N * N * Mx, 0, 0, g.K, 1.0 / N};
        HIP_TRY(c, g.kern->x_fwd3(ax, s));
        // y: [3N][N][Mx] -> [3N][M][Mx]
        ColArgs a{g.C, g.A, g.tw, 3 * N * Mx, Mx, N * Mx, M * Mx, g.K, g.M, 1.0 / N};
        HIP_TRY(c, g.kern->col_fwd(a, s));
        // z + T + Leray: [3][N][MMx] -> compact [3][M][MMx]
        F3Args f{g.A, nullptr, nullptr, g.U1, g.tw, g.rate, g.ones, MMx, (int)MMx, g.Mx, g.K, g.M,
                 0, N * MMx, 0, M * MMx, 0.0, 0.0, 0.0, 1.0 / N};
        HIP_TRY(c, g.kern->f3_proj(f, s));
        HIP_TRY(c, launch_unpack(c->f64, g.U1, uh[i], g.N, g.K, s));
    }
    return NS_OK;
}

ns_status ns_inverse(ns_ctx* c, const void* const* uh, void* const* u)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat")) || (st = check_ptrs(c, (const void* const*)u, "u_phys"))) return st;
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        const long long N = g.N, M = g.M, Mx = g.Mx, MMx = g.MMx;
        hipStream_t s = c->stream;
        HIP_TRY(c, launch_pack(c->f64, uh[i], g.U1, g.N, g.K, s));
        ColArgs a1{g.U1, g.A, g.tw, 3 * MMx, MMx, M * MMx, N * MMx, g.K, g.M, 1.0};
        HIP_TRY(c, g.kern->col_inv(a1, s));
        ColArgs a2{g.A, g.Bw, g.tw, 3 * N * Mx, Mx, M * Mx, N * Mx, g.K, g.M, 1.0};
        HIP_TRY(c, g.kern->col_inv(a2, s));
        XArgs ax{g.Bw, u[i], g.tw, N * N / 2, N * N * Mx, N * N * N, 0, 0, g.K, 1.0};
        HIP_TRY(c, g.kern->x_inv3(ax, s));
    }
    return NS_OK;
}

ns_status ns_rhs(ns_ctx* c, const void* const* uin, void* const* rout)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uin, "uhat_in")) || (st = check_ptrs(c, (const void* const*)rout, "rhs_out"))) return st;
    if ((st = pack_all(c, uin, true))) return st;
    for (Group& g : c->groups)
        if ((st = run_rhs(c, g, g.U0, g.U1, nullptr, 0.0, 0.0, 1.0, g.ones))) return st;
    return unpack_all(c, rout, false);
}

ns_status ns_step(ns_ctx* c, void* const* uh, const double* dt, int32_t nsteps)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, (const void* const*)uh, "uhat"))) return st;
    if ((st = check_dt(c, dt))) return st;
    if (nsteps < 0) return fail(c, NS_ERR_ARG, "nsteps = %d must be >= 0", nsteps);
    if (nsteps == 0) return NS_OK;
    if ((st = pack_all(c, (const void* const*)uh, true))) return st;
    if ((st = set_dt(c, dt))) return st;
    if ((c->prm.flags & NS_USE_GRAPH) && !c->profile) {
        if ((st = ensure_graph(c))) return st;
        for (int i = 0; i < nsteps; ++i) HIP_TRY(c, hipGraphLaunch(c->step_exec, c->stream));
    } else {
        for (int i = 0; i < nsteps; ++i)
            if ((st = step_all(c))) return st;
    }
    if ((st = unpack_all(c, uh, true))) return st;
    if (c->prm.flags & NS_CHECK_FINITE) {
        for (size_t i = 0; i < c->n.size(); ++i) {
            Group& g = c->groups[c->group_of[i]];
            const int kb = std::min(4096, (int)std::ceil(std::sqrt(3.0) * g.K) + 2);
            HIP_TRY(c, launch_spectrum(c->f64, uh[i], c->edev, g.N, g.K, kb, c->stream));
            std::vector<double> E(kb);
            HIP_TRY(c, hipMemcpyAsync(E.data(), c->edev, sizeof(double) * kb, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            double tot = 0;
            for (double e : E) tot += e;
            if (!std::isfinite(tot)) return fail(c, NS_ERR_NONFINITE, "sample %zu: energy is not finite", i);
        }
    }
    return NS_OK;
}

ns_status ns_tape_bytes(const ns_ctx* c, int32_t nsteps, size_t* per)
{
    if (!c || !per || nsteps < 0) return NS_ERR_ARG;
    size_t mx = 0;
    for (const Group& g : c->groups) mx = std::max(mx, (size_t)g.st * 2 * c->rsz * 3);
    *per = mx * (size_t)nsteps;
    return NS_OK;
}

ns_status ns_step_taped(ns_ctx* c, void* const*, const double*, int32_t, void* const*)
{
    CHECK_STATE(c);
    return fail(c, NS_ERR_UNSUPPORTED, "ns_step_taped is not available in this build");
}

ns_status ns_adjoint_step(ns_ctx* c, const void* const*, const void* const*, const double*, void* const*)
{
    CHECK_STATE(c);
    return fail(c, NS_ERR_UNSUPPORTED, "ns_adjoint_step is not available in this build");
}

ns_status ns_energy_spectrum(ns_ctx* c, const void* const* uh, double* E, int32_t kbins)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat"))) return st;
    if (!E || kbins < 1) return fail(c, NS_ERR_ARG, "E must be non-null with kbins >= 1");
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        HIP_TRY(c, launch_spectrum(c->f64, uh[i], E + i * (size_t)kbins, g.N, g.K, kbins, c->stream));
    }
    return NS_OK;
}

}  // extern "C"
