// Host runtime behind the C ABI of include/ns.h: contexts, sample groups,
// workspaces, twiddle and damping tables, the pass sequence of one
// right-hand-side evaluation, SSP-RK3 stages (plain or fused) and hipGraph
// replay, the autotuner, the adjoint, and the in-situ statistics.
#include "../../include/ns.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "args.hpp"
#include "misc_kernels.hpp"

using namespace ns;

namespace ns {
#define NS_SIZES(X) \
    X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(60) X(64) X(80) X(96) X(120) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536)
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
    int L = 0;  // grid of the caller's spectra: N, or 2N/3 for a padded n-mode state
    std::vector<int> samples;  // context sample index of batch slot b
    const SizeKernels* kern = nullptr;
    long long MMx = 0;         // M * Mx, columns of a compact plane
    long long MMxp = 0;        // MMx rounded up to the compact column block
    long long st = 0;          // compact state elements per sample, 3 M MMxp
    int eb = 8;                // bytes per complex element
    double eps = 0, m_cut = 0;
    void *U0 = nullptr, *U1 = nullptr;  // compact states
    void *A = nullptr, *Bw = nullptr, *C = nullptr;  // pass workspaces
    void *tw = nullptr, *rate = nullptr;
    double *dt = nullptr, *ones = nullptr;
    std::vector<double> dt_host;  // values last uploaded to dt
    // adjoint buffers (allocated on first use): stage u2, adjoint stages,
    // and 8-component pass workspaces
    void *U2 = nullptr, *L1 = nullptr, *L2 = nullptr, *L3 = nullptr, *A8 = nullptr, *B8 = nullptr;
    int sel[NS_NPASS] = {0, 0, 0, 0, 0};  // chosen schedule variant per pass
    double tune_ms[NS_NPASS][NS_MAXV] = {};  // tuner timings (ms per launch), 0 = not timed
    // stage form: SSP-RK3 stages end in the fused F3 + inverse z pass (the
    // next stage skips I1); stage_ms: tuner timings of a plain / fused stage
    bool fuse = true;
    double stage_ms[2] = {0.0, 0.0};
    double* zeros = nullptr;  // [B] zero time steps (tuner)
};

enum { FUSE_AUTO = 0, FUSE_OFF = 1, FUSE_ON = 2 };

// variant count / name of pass p (I1 and I2 share the inverse column list)
int variant_count(const SizeKernels* k, int p)
{
    switch (p) {
        case 0:
        case 1: return k->n_inv;
        case 2: return k->n_x;
        case 3: return k->n_fwd;
        default: return k->n_f3;
    }
}

const char* variant_name(const SizeKernels* k, int p, int v)
{
    switch (p) {
        case 0:
        case 1: return k->inv[v].name;
        case 2: return k->x[v].name;
        case 3: return k->fwd[v].name;
        default: return k->f3[v].name;
    }
}

const char* kPassName[NS_NPASS] = {"I1_inv_z", "I2_inv_y", "X_c2r_prod_r2c", "F2_fwd_y", "F3_fwd_z_epilogue"};

}  // namespace

struct ns_ctx {
    ns_params prm{};
    std::vector<int> n;
    std::vector<int> group_of, slot_of;
    bool f64 = false;
    bool pad = false;  // n[i] are mode counts; the passes run on 3n/2 points
    int fuse_mode = 0;  // FUSE_AUTO, FUSE_OFF (NS_NO_FUSE) or FUSE_ON (NS_FUSE)
    size_t rsz = 4;  // bytes per real
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<hipStream_t> branch;     // capture streams of groups 1.. (parallel graph branches)
    std::vector<hipEvent_t> branch_ev;   // fork/join events for the capture
    std::vector<Group> groups;
    std::vector<void*> allocs;
    size_t bytes = 0;
    std::string err;
    bool failed = false;
    hipGraphExec_t step_exec = nullptr;
    hipGraph_t step_graph = nullptr;
    // launch form of the captured step with several size groups: one chain
    // on a single stream, or concurrent branches; graph_ms: their timings
    bool graph_branches = false;
    double graph_ms[2] = {0.0, 0.0};
    std::string tune_cache;
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

// cutoff and compact-layout sizes of a group of grid size g.N
void set_dims(Group& g, bool f64)
{
    g.K = (g.N - 1) / 3;
    g.M = 2 * g.K + 1;
    g.Mx = g.K + 1;
    g.MMx = (long long)g.M * g.Mx;
    g.eb = f64 ? 16 : 8;
    g.MMxp = compact_cols(g.MMx, g.eb);
    g.st = 3LL * g.M * g.MMxp;
}

// column-pass input fields for a compact array of nc components per sample
void compact_in(ColArgs& a, const Group& g, int nc)
{
    const int cb = compact_cb(g.eb);
    a.in_cs = (long long)g.M * cb;
    a.in_ss = (long long)nc * g.M * g.MMxp;
    a.in_bs = (long long)nc * g.M * cb;
    a.in_rs = cb;
    a.in_cbl = compact_cbl(g.eb);
}

ns_status setup_group(ns_ctx* c, Group& g)
{
    const int N = g.N;
    set_dims(g, c->f64);
    g.B = (int)g.samples.size();
    g.kern = find_kernels(N, c->f64);
    if (!g.kern) return fail(c, NS_ERR_UNSUPPORTED, "grid size N=%d is not supported", N);
    const double s = c->prm.s;
    // defaults at the resolution of the state (the mode count when padded)
    g.eps = c->prm.eps >= 0 ? c->prm.eps : 1e-3 * std::pow(32.0 / g.L, 2.0 * s - 1.0);
    g.m_cut = c->prm.m_cut >= 0 ? c->prm.m_cut : g.L / 3.0;
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
    if ((st = dalloc(c, (void**)&g.zeros, sizeof(double) * B))) return st;
    g.fuse = c->fuse_mode != FUSE_OFF;  // the tuner may change it in FUSE_AUTO mode
    for (int v = 0; v < g.kern->n_f3; ++v)
        if (!g.kern->f3[v].fn_zi) return fail(c, NS_ERR_UNSUPPORTED, "N=%d: F3 variant %s has no fused form", N, g.kern->f3[v].name);
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
    std::vector<double> ones(B, 1.0), zeros(B, 0.0);
    if ((st = upload(c, g.ones, ones.data(), sizeof(double) * B))) return st;
    if ((st = upload(c, g.zeros, zeros.data(), sizeof(double) * B))) return st;
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

// Arguments of the five passes of one right-hand-side evaluation for every
// sample of a group: read the compact stage state us (and u0), write
// out = ca u0 + cb us + cc dt F(us).  The I1 output (I2 input) has F2's
// sample stride 6 N MMx, so that the fused F3 + inverse z pass writes it in
// place over the columns it has read.
struct PassArgs {
    ColArgs i1, i2, f2;
    XArgs x;
    F3Args f3;
};

PassArgs pass_args(const Group& g, const void* us, void* out, const void* u0, double ca, double cb, double cc,
                   const double* dt)
{
    const long long N = g.N, B = g.B, M = g.M, Mx = g.Mx, MMx = g.MMx;
    PassArgs a;
    // I1: compact [B][3] -> [B][3 of 6][N][MMx]
    a.i1 = ColArgs{us, g.A, g.tw, B * 3 * MMx, MMx, 3, 0, 0, N * MMx, 6 * N * MMx, g.K, g.M, 1.0};
    compact_in(a.i1, g, 3);
    // I2: [B][3 of 6][N][M][Mx] -> [B*3*N][N][Mx]
    a.i2 = ColArgs{g.A, g.Bw, g.tw, B * 3 * N * Mx, Mx, 3 * N, M * Mx, 6 * N * M * Mx, N * Mx, 3 * N * N * Mx,
                   g.K, g.M, 1.0};
    // X: [B][3][N*N][Mx] -> [B][6][N*N][Mx]
    a.x = XArgs{g.Bw, g.C, g.tw, B * N * N / 2, N * N * Mx, N * N * Mx, 3 * N * N * Mx, 6 * N * N * Mx, g.K, 1.0 / N};
    // F2: [B*6*N][N][Mx] -> [B*6*N][M][Mx]
    a.f2 = ColArgs{g.C, g.A, g.tw, B * 6 * N * Mx, Mx, 6 * N, N * Mx, 6 * N * N * Mx, M * Mx, 6 * N * M * Mx,
                   g.K, g.M, 1.0 / N};
    // F3: [B][6][N][MMx] -> compact [B][3]
    // (the fused form also writes I1 of `out` over its input: [B][3 of 6][N][MMx])
    a.f3 = F3Args{g.A, u0, us, out, g.tw, g.rate, dt, B * g.MMxp, (int)MMx, g.Mx, g.K, g.M,
                  6 * N * MMx, N * MMx, g.st, M * compact_cb(g.eb), ca, cb, cc, 1.0 / N, nullptr, nullptr, 0.0, 0.0, g.A};
    return a;
}

// zi selects the fused F3 + inverse z form of pass 4
hipError_t launch_pass(const Group& g, int p, int v, const PassArgs& a, hipStream_t s, bool zi = false)
{
    const SizeKernels* k = g.kern;
    switch (p) {
        case 0: return k->inv[v].fn(a.i1, s);
        case 1: return k->inv[v].fn(a.i2, s);
        case 2: return k->x[v].fn(a.x, s);
        case 3: return k->fwd[v].fn(a.f2, s);
        default: return zi ? k->f3[v].fn_zi(a.f3, s) : k->f3[v].fn(a.f3, s);
    }
}

ns_status run_rhs(ns_ctx* c, Group& g, const void* us, void* out, const void* u0, double ca, double cb, double cc,
                  const double* dt)
{
    const PassArgs a = pass_args(g, us, out, u0, ca, cb, cc, dt);
    ns_status st;
    for (int p = 0; p < NS_NPASS; ++p)
        if ((st = timed(c, p, [&] { return launch_pass(g, p, g.sel[p], a, c->stream); }))) return st;
    return NS_OK;
}

// First pass of the right-hand side alone: the inverse z transform of us into A.
ns_status run_i1(ns_ctx* c, Group& g, const void* us)
{
    const PassArgs a = pass_args(g, us, nullptr, nullptr, 0.0, 0.0, 0.0, g.dt);
    return timed(c, 0, [&] { return launch_pass(g, 0, g.sel[0], a, c->stream); });
}

// One SSP-RK3 stage out = ca u0 + cb us + cc dt F(us).  With fusion, A holds
// the inverse z transform of us on entry (run_i1, or the previous stage) and
// of out on return, and the stage runs I2, X, F2 and the fused F3; without,
// it is the plain five-pass right-hand side.
ns_status rk3_stage(ns_ctx* c, Group& g, const void* us, void* out, const void* u0, double ca, double cb, double cc)
{
    if (!g.fuse) return run_rhs(c, g, us, out, u0, ca, cb, cc, g.dt);
    const PassArgs a = pass_args(g, us, out, u0, ca, cb, cc, g.dt);
    ns_status st;
    for (int p = 1; p < NS_NPASS; ++p)
        if ((st = timed(c, p, [&] { return launch_pass(g, p, g.sel[p], a, c->stream, true); }))) return st;
    return NS_OK;
}

// Start of a run of fused stages from the state in U0.
ns_status begin_stages(ns_ctx* c, Group& g) { return g.fuse ? run_i1(c, g, g.U0) : NS_OK; }

// One SSP-RK3 step (eq. (2.6)) of a group in place on U0, stages in U1
// (after begin_stages).
ns_status rk3_step(ns_ctx* c, Group& g)
{
    ns_status st;
    // u1 = u + dt F(u)
    if ((st = rk3_stage(c, g, g.U0, g.U1, nullptr, 0.0, 1.0, 1.0))) return st;
    // u2 = 3/4 u + 1/4 u1 + 1/4 dt F(u1)
    if ((st = rk3_stage(c, g, g.U1, g.U1, g.U0, 0.75, 0.25, 0.25))) return st;
    // u^{n+1} = 1/3 u + 2/3 u2 + 2/3 dt F(u2)
    if ((st = rk3_stage(c, g, g.U1, g.U0, g.U0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0))) return st;
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
        HIP_TRY(c, launch_pack(c->f64, uh[i], dst, g.L, g.K, c->stream));
    }
    return NS_OK;
}

ns_status unpack_all(ns_ctx* c, void* const* uh, bool from_u0)
{
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        const char* src = (const char*)(from_u0 ? g.U0 : g.U1) + cwb(c) * g.st * c->slot_of[i];
        HIP_TRY(c, launch_unpack(c->f64, src, uh[i], g.L, g.K, c->stream));
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
        if (v == g.dt_host) continue;  // already on the device
        HIP_TRY(c, hipMemcpyAsync(g.dt, v.data(), sizeof(double) * g.B, hipMemcpyHostToDevice, c->stream));
        // the host vector dies here: wait for the copy
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        g.dt_host = v;
    }
    return NS_OK;
}

// ---------------------------------------------------------------- adjoint
ns_status ensure_adjoint_buffers(ns_ctx* c, Group& g)
{
    if (g.U2) return NS_OK;
    const size_t cw = cwb(c);
    const long long B = g.B, N = g.N;
    ns_status st;
    if ((st = dalloc(c, &g.U2, cw * g.st * B))) return st;
    if ((st = dalloc(c, &g.L1, cw * g.st * B))) return st;
    if ((st = dalloc(c, &g.L2, cw * g.st * B))) return st;
    if ((st = dalloc(c, &g.L3, cw * g.st * B))) return st;
    if ((st = dalloc(c, &g.A8, cw * 8ULL * N * g.MMx * B))) return st;
    if ((st = dalloc(c, &g.B8, cw * 8ULL * N * N * g.Mx * B))) return st;
    return NS_OK;
}

// One vector-Jacobian product of the right-hand side for every sample of a
// group, fused with an adjoint SSP-RK3 stage:
//   out = c3 L3 + c2 L2 + c1 L1 + cc dt (F'(u)^T lam),
//   F'(u)^T lam = T F[2 S(P lam) u] - eps |k|^{2s} Q lam,
// u, lam, L1..L3 and out compact.
ns_status run_vjp(ns_ctx* c, Group& g, const void* u, const void* lam, void* out, double c3, double c2, double c1,
                  double cc, const double* dt)
{
    const SizeKernels* k = g.kern;
    const long long N = g.N, B = g.B, M = g.M, Mx = g.Mx, MMx = g.MMx;
    hipStream_t s = c->stream;
    // the column passes use the schedules chosen for the forward I2, F2
    const auto yinv = k->inv[g.sel[1]].fn, yfwd = k->fwd[g.sel[3]].fn;
    // z: strain of P lam (5 components) and velocity (3), from compact lam
    // and u, -> [B][8][N][MMx]
    const StrainZArgs sz{lam, u, g.A8, g.tw, B * g.MMxp, (int)MMx, g.Mx, g.K, g.M, g.st, M * compact_cb(g.eb),
                         8 * N * MMx, N * MMx};
    HIP_TRY(c, k->strain_z(sz, s));
    // y: [B][8N][M][Mx] -> [B][8N][N][Mx]
    ColArgs y1{g.A8, g.B8, g.tw, B * 8 * N * Mx, Mx, 8 * N, M * Mx, 8 * N * M * Mx, N * Mx, 8 * N * N * Mx,
               g.K, g.M, 1.0};
    HIP_TRY(c, yinv(y1, s));
    // x: a = 2 S u -> [B][3][N*N][Mx]
    XArgs ax{g.B8, g.C, g.tw, B * N * N / 2, N * N * Mx, N * N * Mx, 8 * N * N * Mx, 3 * N * N * Mx, g.K, 1.0 / N};
    HIP_TRY(c, k->x_adj(ax, s));
    // y forward: [B][3N][N][Mx] -> [B][3N][M][Mx]
    ColArgs y2{g.C, g.A, g.tw, B * 3 * N * Mx, Mx, 3 * N, N * Mx, 3 * N * N * Mx, M * Mx, 3 * N * M * Mx,
               g.K, g.M, 1.0 / N};
    HIP_TRY(c, yfwd(y2, s));
    // z forward + adjoint stage epilogue
    F3Args f{g.A, g.L3, lam, out, g.tw, g.rate, dt, B * g.MMxp, (int)MMx, g.Mx, g.K, g.M,
             3 * N * MMx, N * MMx, g.st, M * compact_cb(g.eb), c3, 0.0, cc, 1.0 / N, g.L2, g.L1, c2, c1};
    HIP_TRY(c, k->f3_adj(f, s));
    return NS_OK;
}

// Adjoint of one SSP-RK3 step for a group: stage states u^n, u1, u2 (compact,
// batch-contiguous); lambda_{n+1} in L3 on entry, lambda_n in L3 on return.
ns_status adjoint_rk3(ns_ctx* c, Group& g, const void* un, const void* u1, const void* u2)
{
    ns_status st;
    // lambda_2 = 2/3 lambda_3 + 2/3 dt F'(u2)^T lambda_3
    if ((st = run_vjp(c, g, u2, g.L3, g.L2, 2.0 / 3.0, 0.0, 0.0, 2.0 / 3.0, g.dt))) return st;
    // lambda_1 = 1/4 lambda_2 + 1/4 dt F'(u1)^T lambda_2
    if ((st = run_vjp(c, g, u1, g.L2, g.L1, 0.0, 0.25, 0.0, 0.25, g.dt))) return st;
    // lambda_n = 1/3 lambda_3 + 3/4 lambda_2 + lambda_1 + dt F'(u^n)^T lambda_1
    if ((st = run_vjp(c, g, un, g.L1, g.L3, 1.0 / 3.0, 0.75, 1.0, 1.0, g.dt))) return st;
    return NS_OK;
}

// Stage states of tape step `step` for a group: read in place when the group
// holds one sample (the tape layout is the compact layout), else gathered
// into U0..U2.
ns_status tape_stages(ns_ctx* c, Group& g, const void* const* tape, size_t step_bytes, int step, const void** un,
                      const void** u1, const void** u2)
{
    const size_t one = g.st * 2 * c->rsz;
    if (g.B == 1) {
        const char* base = (const char*)tape[g.samples[0]] + (size_t)step * step_bytes;
        *un = base;
        *u1 = base + one;
        *u2 = base + 2 * one;
        return NS_OK;
    }
    void* dst[3] = {g.U0, g.U1, g.U2};
    for (int b = 0; b < g.B; ++b)
        for (int k = 0; k < 3; ++k)
            HIP_TRY(c, hipMemcpyAsync((char*)dst[k] + b * one,
                                      (const char*)tape[g.samples[b]] + (size_t)step * step_bytes + k * one, one,
                                      hipMemcpyDeviceToDevice, c->stream));
    *un = g.U0;
    *u1 = g.U1;
    *u2 = g.U2;
    return NS_OK;
}

// ---------------------------------------------------------------- autotuner
// Times every schedule variant of each pass on the group's own workspaces
// (filled with seeded random values) and keeps the fastest, then decides the
// stage form: the plain five passes, or I2, X, F2 and the fused F3 + inverse
// z pass, by timing whole stages both ways.  Results are cached per device,
// size, precision and batch in a file of one JSON object per line.
std::string tune_key(const ns_ctx* c, const Group& g)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::ostringstream o;
    o << prop.gcnArchName << "/" << prop.multiProcessorCount << "CU/N=" << g.N << "/" << (c->f64 ? "f64" : "f32")
      << "/B=" << g.B;
    return o.str();
}

std::string json_field(const std::string& line, const char* name)
{
    const std::string key = std::string("\"") + name + "\":\"";
    size_t a = line.find(key);
    if (a == std::string::npos) return "";
    a += key.size();
    size_t b = line.find('"', a);
    return b == std::string::npos ? "" : line.substr(a, b - a);
}

const char* kStageForm = "stage_form";

// Reads the cached choices for key; in FUSE_AUTO mode the stage form must be
// cached too.
bool load_tuning(ns_ctx* c, Group& g, const std::string& path, const std::string& key)
{
    std::ifstream f(path);
    if (!f) return false;
    int found[NS_NPASS] = {-1, -1, -1, -1, -1};
    int form = -1;
    std::string line;
    while (std::getline(f, line)) {
        if (json_field(line, "key") != key) continue;
        const std::string pass = json_field(line, "pass"), var = json_field(line, "variant");
        if (pass == kStageForm) form = var == "fused" ? 1 : (var == "plain" ? 0 : -1);
        for (int p = 0; p < NS_NPASS; ++p) {
            if (pass != kPassName[p]) continue;
            for (int v = 0; v < variant_count(g.kern, p); ++v)
                if (var == variant_name(g.kern, p, v)) found[p] = v;
        }
    }
    for (int p = 0; p < NS_NPASS; ++p)
        if (found[p] < 0) return false;
    if (c->fuse_mode == FUSE_AUTO && form < 0) return false;
    for (int p = 0; p < NS_NPASS; ++p) g.sel[p] = found[p];
    if (c->fuse_mode == FUSE_AUTO) g.fuse = form == 1;
    return true;
}

void save_tuning(const ns_ctx* c, const Group& g, const std::string& path, const std::string& key)
{
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    for (int p = 0; p < NS_NPASS; ++p) {
        const int v = g.sel[p];
        f << "{\"key\":\"" << key << "\",\"pass\":\"" << kPassName[p] << "\",\"variant\":\""
          << variant_name(g.kern, p, v) << "\",\"ms\":" << g.tune_ms[p][v] << "}\n";
    }
    if (c->fuse_mode == FUSE_AUTO)
        f << "{\"key\":\"" << key << "\",\"pass\":\"" << kStageForm << "\",\"variant\":\""
          << (g.fuse ? "fused" : "plain") << "\",\"ms\":" << g.stage_ms[g.fuse ? 1 : 0] << "}\n";
}

ns_status tune_group(ns_ctx* c, Group& g)
{
    const std::string key = tune_key(c, g);
    const char* path = c->tune_cache.empty() ? nullptr : c->tune_cache.c_str();
    if (path && !key.empty() && load_tuning(c, g, path, key)) return NS_OK;
    hipStream_t s = c->stream;
    const size_t cw = cwb(c);
    // the variants are timed on seeded values in [-1, 1) rather than zeros:
    // the x pass draws more power, and runs slower, on realistic data
    const long long per = (long long)(cw / (c->f64 ? 8 : 4));  // reals per complex word
    HIP_TRY(c, launch_fill_random(c->f64, g.U0, per * (long long)g.st * g.B, 1, s));
    HIP_TRY(c, launch_fill_random(c->f64, g.U1, per * (long long)g.st * g.B, 2, s));
    HIP_TRY(c, launch_fill_random(c->f64, g.A, per * 6LL * g.N * g.MMx * g.B, 3, s));
    HIP_TRY(c, launch_fill_random(c->f64, g.Bw, per * 3LL * g.N * g.N * g.Mx * g.B, 4, s));
    HIP_TRY(c, launch_fill_random(c->f64, g.C, per * 6LL * g.N * g.N * g.Mx * g.B, 5, s));
    PassArgs a = pass_args(g, g.U0, g.U1, g.U0, 0.75, 0.25, 0.25, g.ones);
    // single F3 launches write their fused output to C, so that repeated
    // launches do not feed on their own results
    a.f3.zinv = g.C;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    // device time per call of launch(): one warm-up call, one timed call to
    // size the repetitions (about 20 ms in all), then the timed repetitions
    auto time_it = [&](auto&& launch, double& out_ms) -> hipError_t {
        hipError_t e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms1 = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms1, e0, e1);
        const int reps = ms1 > 0 ? (int)std::min(20.0, std::max(2.0, 20.0 / ms1)) : 2;
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        out_ms = ms / reps;
        return e;
    };
    ns_status st = NS_OK;
    // F3 forms to time: 0 = plain, 1 = fused
    const bool forms[2] = {c->fuse_mode != FUSE_ON, c->fuse_mode != FUSE_OFF};
    int best_f3[2] = {0, 0};
    double f3_ms[2][NS_MAXV] = {};
    for (int p = 0; p < NS_NPASS && st == NS_OK; ++p) {
        const int nv = variant_count(g.kern, p);
        for (int zi = 0; zi < 2 && st == NS_OK; ++zi) {
            if (zi == 1 && p != 4) break;
            if (p == 4 && !forms[zi]) continue;
            int best = 0;
            double best_ms = 1e300;
            for (int v = 0; v < nv && nv > 1; ++v) {
                double ms = 0.0;
                const hipError_t e = time_it([&] { return launch_pass(g, p, v, a, s, zi == 1); }, ms);
                if (e != hipSuccess) {
                    st = fail(c, NS_ERR_HIP, "tuning pass %s variant %s failed: %s", kPassName[p],
                              variant_name(g.kern, p, v), hipGetErrorString(e));
                    break;
                }
                if (p == 4) f3_ms[zi][v] = ms;
                else g.tune_ms[p][v] = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = v;
                }
            }
            if (p == 4) best_f3[zi] = best;
            else g.sel[p] = best;
        }
    }
    // whole stages both ways, with dt = 0 (out = us, so that repetitions
    // keep their values) and the fused output in place as in a step
    if (st == NS_OK && c->fuse_mode == FUSE_AUTO) {
        const PassArgs sa = pass_args(g, g.U0, g.U1, g.U0, 0.75, 0.25, 0.25, g.zeros);
        auto stage = [&](int zi) -> hipError_t {
            hipError_t e = hipSuccess;
            for (int p = zi ? 1 : 0; p < NS_NPASS && e == hipSuccess; ++p)
                e = launch_pass(g, p, p == 4 ? best_f3[zi] : g.sel[p], sa, s, zi == 1);
            return e;
        };
        g.stage_ms[0] = g.stage_ms[1] = 1e300;
        for (int r = 0; r < 4 && st == NS_OK; ++r) {  // alternated, best of two each
            const int zi = r & 1;
            double ms = 0.0;
            const hipError_t e = time_it([&] { return stage(zi); }, ms);
            if (e != hipSuccess) st = fail(c, NS_ERR_HIP, "timing the stage forms failed: %s", hipGetErrorString(e));
            g.stage_ms[zi] = std::min(g.stage_ms[zi], ms);
        }
        // the fused form must win by more than 1 %: within timing noise the
        // plain form is kept, so that the choice does not flip between runs
        g.fuse = g.stage_ms[1] < 0.99 * g.stage_ms[0];
    }
    const int form = g.fuse ? 1 : 0;
    g.sel[4] = best_f3[form];
    for (int v = 0; v < NS_MAXV; ++v) g.tune_ms[4][v] = f3_ms[form][v];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == NS_OK && path && !key.empty()) save_tuning(c, g, path, key);
    return st;
}

// One SSP-RK3 step of all groups captured as a graph.  As a chain, every
// group runs on the capture stream in turn.  As branches, group 0 runs on
// the capture stream and every further group on a branch stream forked from
// it and joined back, so groups of different N run concurrently on replay.
ns_status capture_step(ns_ctx* c)
{
    const size_t ng = c->graph_branches ? c->groups.size() : 1;
    hipStream_t main = c->cap_stream;
    ns_status st = NS_OK;
    if (!c->graph_branches) {
        c->stream = main;
        for (Group& g : c->groups)
            if ((st = rk3_step(c, g))) return st;
        return NS_OK;
    }
    if (ng > 1) {
        HIP_TRY(c, hipEventRecord(c->branch_ev[0], main));
        for (size_t g = 1; g < ng; ++g) HIP_TRY(c, hipStreamWaitEvent(c->branch[g - 1], c->branch_ev[0], 0));
    }
    for (size_t g = 0; g < ng && st == NS_OK; ++g) {
        c->stream = g == 0 ? main : c->branch[g - 1];
        st = rk3_step(c, c->groups[g]);
    }
    c->stream = main;
    if (st) return st;
    for (size_t g = 1; g < ng; ++g) {
        HIP_TRY(c, hipEventRecord(c->branch_ev[g], c->branch[g - 1]));
        HIP_TRY(c, hipStreamWaitEvent(main, c->branch_ev[g], 0));
    }
    return NS_OK;
}

ns_status ensure_graph(ns_ctx* c)
{
    if (c->step_exec) return NS_OK;
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    while (c->branch.size() + 1 < c->groups.size()) {
        hipStream_t b = nullptr;
        HIP_TRY(c, hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
        c->branch.push_back(b);
    }
    while (c->branch_ev.size() < c->groups.size()) {
        hipEvent_t e = nullptr;
        HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->branch_ev.push_back(e);
    }
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->stream = user;
        return fail(c, NS_ERR_HIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    }
    ns_status st = capture_step(c);
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

ns_status drop_graph(ns_ctx* c)
{
    if (!c->step_exec) return NS_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    (void)hipGraphExecDestroy(c->step_exec);
    (void)hipGraphDestroy(c->step_graph);
    c->step_exec = nullptr;
    c->step_graph = nullptr;
    return NS_OK;
}

// The launch form of the captured step with several size groups, timed both
// ways on seeded states with dt = 0 (alternated, best of two each).  The
// branches are kept only if they win by more than 1 %: groups that each
// saturate HBM gain nothing from running side by side.  The states are left
// holding the seeded values; every stepping call packs its input first.
ns_status tune_graph_form(ns_ctx* c)
{
    hipStream_t s = c->stream;
    const long long per = (long long)(cwb(c) / c->rsz);  // reals per complex word
    for (Group& g : c->groups) {
        HIP_TRY(c, launch_fill_random(c->f64, g.U0, per * (long long)g.st * g.B, 1, s));
        HIP_TRY(c, launch_fill(g.dt, 0.0, g.B, s));
        g.dt_host.clear();  // the next set_dt uploads the caller's steps
        ns_status st = begin_stages(c, g);
        if (st) return st;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    ns_status st = NS_OK;
    double best[2] = {1e300, 1e300};
    for (int r = 0; r < 4 && st == NS_OK; ++r) {
        c->graph_branches = (r & 1) != 0;
        if ((st = drop_graph(c)) || (st = ensure_graph(c))) break;
        hipError_t e = hipGraphLaunch(c->step_exec, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipGraphLaunch(c->step_exec, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) st = fail(c, NS_ERR_HIP, "timing the graph forms failed: %s", hipGetErrorString(e));
        best[r & 1] = std::min(best[r & 1], ms / 3.0);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    c->graph_ms[0] = best[0];
    c->graph_ms[1] = best[1];
    const bool branches = best[1] < 0.99 * best[0];
    if (branches != c->graph_branches) {
        c->graph_branches = branches;
        return drop_graph(c);
    }
    return NS_OK;
}


// ---------------------------------------------------------------- allocation-free right-hand side
// Workspaces of ns_rhs_noalloc: one static array per GPU.  Host code uses the
// device address that hipGetSymbolAddress returns for the current device
// (scratch_ptr), never the array's own name.
static __device__ __align__(256) unsigned char scratch[NS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct ScratchState {
    void* ptr = nullptr;  // device address of scratch on this GPU
    // parameters of the tables the array holds (valid = uploaded)
    bool valid = false, f64 = false;
    int N = 0, L = 0, q_kind = 0;
    double eps = 0, s = 0, m_cut = 0, theta = 0;
};
std::mutex g_scratch_mu;
ScratchState g_scratch[kMaxDevices];

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Byte offsets of the regions of one sample's workspaces in the array.
struct ScratchLayout {
    size_t U0, U1, A, Bw, C, tw, rate, one, end;
};

ScratchLayout scratch_layout(const Group& g, size_t rsz)
{
    const size_t cw = 2 * rsz, N = g.N;
    ScratchLayout l{};
    size_t o = 0;
    l.U0 = o;
    o += align256(cw * g.st);
    l.U1 = o;
    o += align256(cw * g.st);
    l.A = o;
    o += align256(cw * 6 * N * g.MMx);
    l.Bw = o;
    o += align256(cw * 3 * N * N * g.Mx);
    l.C = o;
    o += align256(cw * 6 * N * N * g.Mx);
    l.tw = o;
    o += align256(cw * N);
    l.rate = o;
    o += align256(rsz * (3 * (size_t)g.K * g.K + 1));
    l.one = o;
    o += align256(sizeof(double));
    l.end = o;
    return l;
}

ns_status noalloc_fail(ns_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_init_error = buf;
    return st;
}

#define NOALLOC_TRY(expr)                                                                                        \
    do {                                                                                                         \
        hipError_t e_ = (expr);                                                                                  \
        if (e_ != hipSuccess) return noalloc_fail(NS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Uploads the twiddle and damping tables of g (and the unit time step) into
// the array at base.  The host tables are stack buffers, so the upload waits
// for the copies before it returns.
template <typename R>
ns_status noalloc_tables(const Group& g, const ns_params* p, char* base, const ScratchLayout& l, hipStream_t s)
{
    // every grid whose workspaces fit the array is far below these bounds
    constexpr int kMaxN = 128, kMaxRate = 3 * 42 * 42 + 1;
    if (g.N > kMaxN || 3 * g.K * g.K + 1 > kMaxRate) return noalloc_fail(NS_ERR_ARG, "N=%d is too large", g.N);
    R tw[2 * kMaxN];
    R rt[kMaxRate];
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int e = 0; e < g.N; ++e) {
        const long double a = 2.0L * pi * (long double)e / (long double)g.N;
        tw[2 * e] = (R)cosl(a);
        tw[2 * e + 1] = (R)(-sinl(a));
    }
    const int nr = 3 * g.K * g.K + 1;
    for (int k2 = 0; k2 < nr; ++k2) {
        const double kabs = std::sqrt((double)k2);
        double q;
        if (kabs <= g.m_cut) q = 0.0;
        else if (p->q_kind == 0) q = 1.0;
        else q = 1.0 - std::pow(g.m_cut / kabs, (2.0 * p->s - 1.0) / p->theta);
        rt[k2] = (R)(g.eps * std::pow((double)k2, p->s) * q);
    }
    NOALLOC_TRY(hipMemcpyAsync(base + l.tw, tw, sizeof(R) * 2 * g.N, hipMemcpyHostToDevice, s));
    NOALLOC_TRY(hipMemcpyAsync(base + l.rate, rt, sizeof(R) * nr, hipMemcpyHostToDevice, s));
    NOALLOC_TRY(launch_fill(reinterpret_cast<double*>(base + l.one), 1.0, 1, s));
    NOALLOC_TRY(hipStreamSynchronize(s));
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
    if ((p->flags & NS_NO_FUSE) && (p->flags & NS_FUSE))
        return fail(nullptr, NS_ERR_ARG, "NS_FUSE and NS_NO_FUSE exclude each other");
    if ((p->flags & NS_GRAPH_CHAIN) && (p->flags & NS_GRAPH_BRANCHES))
        return fail(nullptr, NS_ERR_ARG, "NS_GRAPH_CHAIN and NS_GRAPH_BRANCHES exclude each other");
    const bool pad = (p->flags & NS_PAD) != 0;
    for (int i = 0; i < p->nsamples; ++i) {
        if (pad && (p->n[i] < 8 || p->n[i] % 2 != 0 || !find_kernels(3 * p->n[i] / 2, p->dtype == NS_F64)))
            return fail(nullptr, NS_ERR_UNSUPPORTED, "padded state of n[%d]=%d modes: grid %d is not supported", i,
                        p->n[i], 3 * p->n[i] / 2);
        if (!pad && !find_kernels(p->n[i], p->dtype == NS_F64))
            return fail(nullptr, NS_ERR_UNSUPPORTED, "grid size n[%d]=%d is not supported", i, p->n[i]);
    }
    ns_ctx* c = new ns_ctx;
    c->prm = *p;
    c->prm.n = nullptr;
    c->prm.tune_cache = nullptr;
    if (p->tune_cache) c->tune_cache = p->tune_cache;
    c->f64 = p->dtype == NS_F64;
    c->pad = pad;
    c->fuse_mode = (p->flags & NS_NO_FUSE) ? FUSE_OFF : ((p->flags & NS_FUSE) ? FUSE_ON : FUSE_AUTO);
    c->rsz = c->f64 ? 8 : 4;
    c->stream = (hipStream_t)hip_stream;
    c->n.assign(p->n, p->n + p->nsamples);
    c->group_of.resize(c->n.size());
    c->slot_of.resize(c->n.size());
    for (size_t i = 0; i < c->n.size(); ++i) {
        int gi = -1;
        for (size_t j = 0; j < c->groups.size(); ++j)
            if (c->groups[j].L == c->n[i]) gi = (int)j;
        if (gi < 0) {
            c->groups.emplace_back();
            c->groups.back().L = c->n[i];
            c->groups.back().N = pad ? 3 * c->n[i] / 2 : c->n[i];
            gi = (int)c->groups.size() - 1;
        }
        c->group_of[i] = gi;
        c->slot_of[i] = (int)c->groups[gi].samples.size();
        c->groups[gi].samples.push_back((int)i);
    }
    ns_status st = NS_OK;
    for (Group& g : c->groups)
        if ((st = setup_group(c, g))) break;
    if (st == NS_OK && !(p->flags & NS_NO_TUNE))
        for (Group& g : c->groups)
            if ((st = tune_group(c, g))) break;
    c->graph_branches = (p->flags & NS_GRAPH_BRANCHES) != 0;
    if (st == NS_OK && (p->flags & NS_USE_GRAPH) && c->groups.size() > 1 && !(p->flags & NS_NO_TUNE)
        && !(p->flags & (NS_GRAPH_CHAIN | NS_GRAPH_BRANCHES)))
        st = tune_graph_form(c);
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
    for (hipStream_t b : c->branch) (void)hipStreamDestroy(b);
    for (hipEvent_t e : c->branch_ev) (void)hipEventDestroy(e);
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

// the group of the samples of size n (the mode count when padded)
static Group* group_of_size(ns_ctx* c, int n)
{
    for (Group& g : c->groups)
        if (g.L == n) return &g;
    return nullptr;
}

ns_status ns_variant_count(ns_ctx* c, int32_t n, int32_t pass, int32_t* count)
{
    CHECK_STATE(c);
    Group* g = group_of_size(c, n);
    if (!g || pass < 0 || pass >= NS_NPASS || !count) return fail(c, NS_ERR_ARG, "no samples of size %d or bad pass", n);
    *count = variant_count(g->kern, pass);
    return NS_OK;
}

ns_status ns_set_variant(ns_ctx* c, int32_t n, int32_t pass, int32_t variant)
{
    CHECK_STATE(c);
    Group* g = group_of_size(c, n);
    if (!g || pass < 0 || pass >= NS_NPASS) return fail(c, NS_ERR_ARG, "no samples of size %d or bad pass", n);
    if (variant < 0 || variant >= variant_count(g->kern, pass))
        return fail(c, NS_ERR_ARG, "variant %d out of range for pass %d at N=%d", variant, pass, n);
    g->sel[pass] = variant;
    return drop_graph(c);  // the captured step used the old schedule
}

ns_status ns_tune_report(ns_ctx* c, char* buf, size_t len, size_t* needed)
{
    CHECK_STATE(c);
    std::ostringstream o;
    o << "[";
    bool first = true;
    for (const Group& g : c->groups) {
        for (int p = 0; p < NS_NPASS; ++p) {
            if (!first) o << ",";
            first = false;
            o << "{\"N\":" << g.L << ",\"grid\":" << g.N << ",\"batch\":" << g.B << ",\"pass\":\"" << kPassName[p] << "\",\"selected\":\""
              << variant_name(g.kern, p, g.sel[p]) << "\",\"timings_ms\":{";
            for (int v = 0; v < variant_count(g.kern, p); ++v)
                o << (v ? "," : "") << "\"" << variant_name(g.kern, p, v) << "\":" << g.tune_ms[p][v];
            o << "}";
            // the stage form, on the F3 entry (its timings are of that form)
            if (p == 4)
                o << ",\"fused\":" << (g.fuse ? "true" : "false") << ",\"stage_ms\":{\"plain\":" << g.stage_ms[0]
                  << ",\"fused\":" << g.stage_ms[1] << "}";
            if (p == 4 && c->groups.size() > 1)
                o << ",\"graph_form\":\"" << (c->graph_branches ? "branches" : "chain") << "\",\"graph_ms\":{\"chain\":"
                  << c->graph_ms[0] << ",\"branches\":" << c->graph_ms[1] << "}";
            o << "}";
        }
    }
    o << "]";
    const std::string r = o.str();
    if (needed) *needed = r.size() + 1;
    if (buf && len > 0) {
        const size_t m = std::min(len - 1, r.size());
        memcpy(buf, r.data(), m);
        buf[m] = 0;
    }
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
        HIP_TRY(c, launch_project(c->f64, uh[i], g.L, g.K, c->stream));
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
        ColArgs a{g.C, g.A, g.tw, 3 * N * Mx, Mx, 3 * N, N * Mx, 3 * N * N * Mx, M * Mx, 3 * N * M * Mx,
                  g.K, g.M, 1.0 / N};
        HIP_TRY(c, g.kern->fwd[g.sel[3]].fn(a, s));
        // z + T + Leray: [3][N][MMx] -> compact [3]
        F3Args f{g.A, nullptr, nullptr, g.U1, g.tw, g.rate, g.ones, g.MMxp, (int)MMx, g.Mx, g.K, g.M,
                 0, N * MMx, 0, M * compact_cb(g.eb), 0.0, 0.0, 0.0, 1.0 / N, nullptr, nullptr, 0.0, 0.0};
        HIP_TRY(c, g.kern->f3_proj(f, s));
        HIP_TRY(c, launch_unpack(c->f64, g.U1, uh[i], g.L, g.K, s));
    }
    return NS_OK;
}

// Physical field u = F^-1[T uhat] of one sample of group g into u ([3][N^3]
// reals); uses U1, A and Bw as workspaces.
static ns_status inverse_one(ns_ctx* c, Group& g, const void* uh, void* u)
{
    const long long N = g.N, M = g.M, Mx = g.Mx, MMx = g.MMx;
    hipStream_t s = c->stream;
    HIP_TRY(c, launch_pack(c->f64, uh, g.U1, g.L, g.K, s));
    ColArgs a1{g.U1, g.A, g.tw, 3 * MMx, MMx, 3, 0, 0, N * MMx, 3 * N * MMx, g.K, g.M, 1.0};
    compact_in(a1, g, 3);
    HIP_TRY(c, g.kern->inv[g.sel[0]].fn(a1, s));
    ColArgs a2{g.A, g.Bw, g.tw, 3 * N * Mx, Mx, 3 * N, M * Mx, 3 * N * M * Mx, N * Mx, 3 * N * N * Mx,
               g.K, g.M, 1.0};
    HIP_TRY(c, g.kern->inv[g.sel[1]].fn(a2, s));
    XArgs ax{g.Bw, u, g.tw, N * N / 2, N * N * Mx, N * N * N, 0, 0, g.K, 1.0};
    HIP_TRY(c, g.kern->x_inv3(ax, s));
    return NS_OK;
}

// The physical fields of every sample of group g into C ([B][3][N^3]
// reals; C holds 4 N^3 B or more) in three batched passes: compact states
// in U1, I1 and I2 as in a right-hand side, then the C2R of all samples.
static ns_status group_to_grid(ns_ctx* c, Group& g, const void* const* uh)
{
    const long long N = g.N, B = g.B, Mx = g.Mx;
    hipStream_t s = c->stream;
    for (int b = 0; b < g.B; ++b)
        HIP_TRY(c, launch_pack(c->f64, uh[g.samples[b]], (char*)g.U1 + cwb(c) * g.st * b, g.L, g.K, s));
    const PassArgs a = pass_args(g, g.U1, nullptr, nullptr, 0.0, 0.0, 0.0, g.dt);
    HIP_TRY(c, launch_pass(g, 0, g.sel[0], a, s));
    HIP_TRY(c, launch_pass(g, 1, g.sel[1], a, s));
    XArgs ax{g.Bw, g.C, g.tw, B * N * N / 2, N * N * Mx, N * N * N, 3 * N * N * Mx, 3 * N * N * N, g.K, 1.0};
    HIP_TRY(c, g.kern->x_inv3(ax, s));
    return NS_OK;
}

ns_status ns_inverse(ns_ctx* c, const void* const* uh, void* const* u)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat")) || (st = check_ptrs(c, (const void* const*)u, "u_phys"))) return st;
    for (size_t i = 0; i < c->n.size(); ++i)
        if ((st = inverse_one(c, c->groups[c->group_of[i]], uh[i], u[i]))) return st;
    return NS_OK;
}

ns_status ns_moments(ns_ctx* c, const void* const* uh, int32_t n, double* mean, double* var)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat"))) return st;
    if (!mean || !var || mean == var) return fail(c, NS_ERR_ARG, "mean and var must be distinct non-null device arrays");
    Group* gp = group_of_size(c, n);
    if (!gp) return fail(c, NS_ERR_ARG, "no samples of size %d", n);
    Group& g = *gp;
    const long long N = g.N;
    if ((st = group_to_grid(c, g, uh))) return st;
    HIP_TRY(c, launch_moments(c->f64, g.C, g.B, 3LL * N * N * N, mean, var, c->stream));
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
    for (Group& g : c->groups)
        if ((st = begin_stages(c, g))) return st;
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
            HIP_TRY(c, launch_spectrum(c->f64, uh[i], c->edev, g.L, g.K, kb, c->stream));
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

// tape layout per sample: [step][stage u^n, u1, u2][compact state]
static size_t tape_step_bytes(const ns_ctx* c, const Group& g) { return (size_t)g.st * 2 * c->rsz * 3; }

ns_status ns_tape_step_bytes(const ns_ctx* c, int32_t n, size_t* bytes)
{
    if (!c || !bytes) return NS_ERR_ARG;
    for (const Group& g : c->groups)
        if (g.L == n) {
            *bytes = tape_step_bytes(c, g);
            return NS_OK;
        }
    return NS_ERR_ARG;
}

ns_status ns_step_taped(ns_ctx* c, void* const* uh, const double* dt, int32_t nsteps, void* const* tape)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, (const void* const*)uh, "uhat")) || (st = check_ptrs(c, (const void* const*)tape, "tape")))
        return st;
    if ((st = check_dt(c, dt))) return st;
    if (nsteps < 0) return fail(c, NS_ERR_ARG, "nsteps = %d must be >= 0", nsteps);
    if (nsteps == 0) return NS_OK;
    if ((st = pack_all(c, (const void* const*)uh, true))) return st;
    if ((st = set_dt(c, dt))) return st;
    for (Group& g : c->groups)
        if ((st = begin_stages(c, g))) return st;
    const size_t sb = 2 * c->rsz;
    for (int n = 0; n < nsteps; ++n) {
        for (Group& g : c->groups) {
            const size_t one = g.st * sb, step = tape_step_bytes(c, g);
            auto save = [&](const void* src, int stage) -> ns_status {
                for (int b = 0; b < g.B; ++b) {
                    char* dst = (char*)tape[g.samples[b]] + (size_t)n * step + (size_t)stage * one;
                    HIP_TRY(c, hipMemcpyAsync(dst, (const char*)src + b * one, one, hipMemcpyDeviceToDevice, c->stream));
                }
                return NS_OK;
            };
            // the stages of rk3_step, with the stage states saved in between
            if ((st = save(g.U0, 0))) return st;
            if ((st = rk3_stage(c, g, g.U0, g.U1, nullptr, 0.0, 1.0, 1.0))) return st;
            if ((st = save(g.U1, 1))) return st;
            if ((st = rk3_stage(c, g, g.U1, g.U1, g.U0, 0.75, 0.25, 0.25))) return st;
            if ((st = save(g.U1, 2))) return st;
            if ((st = rk3_stage(c, g, g.U1, g.U0, g.U0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0))) return st;
        }
    }
    return unpack_all(c, uh, true);
}

ns_status ns_adjoint_step(ns_ctx* c, const void* const* uh, const void* const* tape_step, const double* dt,
                          void* const* lam)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, (const void* const*)lam, "lam")) || (st = check_dt(c, dt))) return st;
    if (tape_step) {
        if ((st = check_ptrs(c, tape_step, "tape_step"))) return st;
    } else if ((st = check_ptrs(c, uh, "uhat_n"))) {
        return st;
    }
    for (Group& g : c->groups)
        if ((st = ensure_adjoint_buffers(c, g))) return st;
    if ((st = set_dt(c, dt))) return st;
    const size_t sb = 2 * c->rsz;
    for (Group& g : c->groups) {
        const size_t one = g.st * sb;
        const void *un = g.U0, *u1 = g.U1, *u2 = g.U2;
        if (tape_step) {
            if ((st = tape_stages(c, g, tape_step, 0, 0, &un, &u1, &u2))) return st;
        } else {
            for (int b = 0; b < g.B; ++b)
                HIP_TRY(c, launch_pack(c->f64, uh[g.samples[b]], (char*)g.U0 + b * one, g.L, g.K, c->stream));
            // the first two stages exactly as ns_step_taped computes them
            if ((st = begin_stages(c, g))) return st;
            if ((st = rk3_stage(c, g, g.U0, g.U1, nullptr, 0.0, 1.0, 1.0))) return st;
            if ((st = rk3_stage(c, g, g.U1, g.U2, g.U0, 0.75, 0.25, 0.25))) return st;
        }
        for (int b = 0; b < g.B; ++b)
            HIP_TRY(c, launch_pack(c->f64, lam[g.samples[b]], (char*)g.L3 + b * one, g.L, g.K, c->stream));
        if ((st = adjoint_rk3(c, g, un, u1, u2))) return st;
        for (int b = 0; b < g.B; ++b)
            HIP_TRY(c, launch_unpack(c->f64, (const char*)g.L3 + b * one, lam[g.samples[b]], g.L, g.K, c->stream));
    }
    return NS_OK;
}

ns_status ns_adjoint_steps(ns_ctx* c, const void* const* tape, int32_t nsteps, const double* dt, void* const* lam)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, (const void* const*)lam, "lam")) || (st = check_ptrs(c, tape, "tape")) ||
        (st = check_dt(c, dt)))
        return st;
    if (nsteps < 0) return fail(c, NS_ERR_ARG, "nsteps = %d must be >= 0", nsteps);
    if (nsteps == 0) return NS_OK;
    for (Group& g : c->groups)
        if ((st = ensure_adjoint_buffers(c, g))) return st;
    if ((st = set_dt(c, dt))) return st;
    const size_t sb = 2 * c->rsz;
    for (Group& g : c->groups) {
        const size_t one = g.st * sb;
        for (int b = 0; b < g.B; ++b)
            HIP_TRY(c, launch_pack(c->f64, lam[g.samples[b]], (char*)g.L3 + b * one, g.L, g.K, c->stream));
        for (int step = nsteps - 1; step >= 0; --step) {
            const void *un, *u1, *u2;
            if ((st = tape_stages(c, g, tape, tape_step_bytes(c, g), step, &un, &u1, &u2))) return st;
            if ((st = adjoint_rk3(c, g, un, u1, u2))) return st;
        }
        for (int b = 0; b < g.B; ++b)
            HIP_TRY(c, launch_unpack(c->f64, (const char*)g.L3 + b * one, lam[g.samples[b]], g.L, g.K, c->stream));
    }
    return NS_OK;
}

ns_status ns_structure_functions(ns_ctx* c, const void* const* uh, int32_t lmax, double p, double* S)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat"))) return st;
    if (!S || !(p > 0) || !std::isfinite(p)) return fail(c, NS_ERR_ARG, "S must be non-null and p finite and > 0");
    for (Group& g : c->groups) {
        if (lmax < 1 || lmax > g.N / 2) return fail(c, NS_ERR_ARG, "lmax = %d must lie in 1..%d", lmax, g.N / 2);
        // the partial sums go to A, free once the fields are in C
        const size_t need = sizeof(double) * (size_t)sfun_blocks(g.N) * lmax * g.B;
        if (need > cwb(c) * 6ULL * g.N * g.MMx * g.B)
            return fail(c, NS_ERR_ARG, "lmax = %d needs more scratch than the workspace holds", lmax);
    }
    for (Group& g : c->groups) {
        if ((st = group_to_grid(c, g, uh))) return st;
        double* part = (double*)g.A;
        HIP_TRY(c, launch_sfun(c->f64, g.C, g.N, lmax, g.B, p, part, c->stream));
        const size_t per = (size_t)sfun_blocks(g.N) * lmax;
        for (int b = 0; b < g.B; ++b)
            HIP_TRY(c, launch_sfun_final(part + b * per, g.N, lmax, S + (size_t)g.samples[b] * lmax, c->stream));
    }
    return NS_OK;
}

ns_status ns_wasserstein1(ns_ctx* c, const void* a, int32_t na, const void* b, int32_t nb, int32_t n, double* w,
                          double* mean)
{
    CHECK_STATE(c);
    if (!a || !b || !w) return fail(c, NS_ERR_ARG, "a, b and w must be non-null device arrays");
    if (na < 1 || nb < 1 || n < 1) return fail(c, NS_ERR_ARG, "na = %d, nb = %d and n = %d must be >= 1", na, nb, n);
    if (na + nb > 20480) return fail(c, NS_ERR_ARG, "na + nb = %d exceeds 20480", na + nb);
    HIP_TRY(c, launch_w1(c->f64, a, na, b, nb, 3LL * n * n * n, 3, w, mean, c->stream));
    return NS_OK;
}

static ns_status spectrum_all(ns_ctx* c, const void* const* uh, double* E, int32_t kbins, int kind)
{
    CHECK_STATE(c);
    ns_status st;
    if ((st = check_ptrs(c, uh, "uhat"))) return st;
    if (!E || kbins < 1) return fail(c, NS_ERR_ARG, "E must be non-null with kbins >= 1");
    for (size_t i = 0; i < c->n.size(); ++i) {
        Group& g = c->groups[c->group_of[i]];
        HIP_TRY(c, launch_spectrum(c->f64, uh[i], E + i * (size_t)kbins, g.L, g.K, kbins, c->stream, kind));
    }
    return NS_OK;
}

ns_status ns_energy_spectrum(ns_ctx* c, const void* const* uh, double* E, int32_t kbins)
{
    return spectrum_all(c, uh, E, kbins, 0);
}

ns_status ns_enstrophy_spectrum(ns_ctx* c, const void* const* uh, double* Z, int32_t kbins)
{
    return spectrum_all(c, uh, Z, kbins, 1);
}


ns_status ns_rhs_noalloc(const ns_params* p, const void* uin, void* rout, void* hip_stream)
{
    if (!p) return noalloc_fail(NS_ERR_ARG, "params is null");
    if (p->dtype != NS_F32 && p->dtype != NS_F64) return noalloc_fail(NS_ERR_ARG, "bad dtype %d", (int)p->dtype);
    if (p->nsamples != 1 || !p->n) return noalloc_fail(NS_ERR_ARG, "ns_rhs_noalloc takes one sample (nsamples = 1)");
    if (!uin || !rout) return noalloc_fail(NS_ERR_ARG, "uhat_in and rhs_out must be non-null");
    if (uin == rout) return noalloc_fail(NS_ERR_ARG, "uhat_in and rhs_out may not alias");
    if (!(p->s >= 0) || !std::isfinite(p->s)) return noalloc_fail(NS_ERR_ARG, "s must be finite and >= 0");
    if (p->q_kind != 0 && p->q_kind != 1) return noalloc_fail(NS_ERR_ARG, "q_kind must be 0 or 1");
    if (p->q_kind == 1 && !(p->theta > 0)) return noalloc_fail(NS_ERR_ARG, "theta must be > 0 for q_kind 1");
    if (!std::isfinite(p->eps) || !std::isfinite(p->m_cut)) return noalloc_fail(NS_ERR_ARG, "eps and m_cut must be finite");
    const bool f64 = p->dtype == NS_F64, pad = (p->flags & NS_PAD) != 0;
    const int L = p->n[0];
    if (pad && (L < 8 || L % 2 != 0)) return noalloc_fail(NS_ERR_UNSUPPORTED, "padded state of n=%d modes is not supported", L);
    Group g;  // describes the sample; its buffers are regions of the array
    g.L = L;
    g.N = pad ? 3 * L / 2 : L;
    g.kern = find_kernels(g.N, f64);
    if (!g.kern) return noalloc_fail(NS_ERR_UNSUPPORTED, "grid size N=%d is not supported", g.N);
    set_dims(g, f64);
    g.B = 1;
    g.eps = p->eps >= 0 ? p->eps : 1e-3 * std::pow(32.0 / g.L, 2.0 * p->s - 1.0);
    g.m_cut = p->m_cut >= 0 ? p->m_cut : g.L / 3.0;
    const size_t rsz = f64 ? 8 : 4;
    const ScratchLayout l = scratch_layout(g, rsz);
    if (l.end > NS_NOALLOC_SCRATCH_BYTES)
        return noalloc_fail(NS_ERR_ARG, "grid N=%d (%s) needs %zu bytes of scratch; the static array holds %zu", g.N,
                            f64 ? "FP64" : "FP32", l.end, (size_t)NS_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    NOALLOC_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return noalloc_fail(NS_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    hipStream_t s = (hipStream_t)hip_stream;
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ScratchState& ss = g_scratch[dev];
        if (!ss.ptr) {
            void* ptr = nullptr;
            NOALLOC_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return noalloc_fail(NS_ERR_HIP, "hipGetSymbolAddress returned a null address");
            ss.ptr = ptr;
        }
        base = static_cast<char*>(ss.ptr);
        const bool same = ss.valid && ss.f64 == f64 && ss.N == g.N && ss.L == g.L && ss.q_kind == p->q_kind &&
                          ss.eps == g.eps && ss.s == p->s && ss.m_cut == g.m_cut && ss.theta == p->theta;
        if (!same) {
            ss.valid = false;
            const ns_status st = f64 ? noalloc_tables<double>(g, p, base, l, s) : noalloc_tables<float>(g, p, base, l, s);
            if (st) return st;
            ss.valid = true;
            ss.f64 = f64;
            ss.N = g.N;
            ss.L = g.L;
            ss.q_kind = p->q_kind;
            ss.eps = g.eps;
            ss.s = p->s;
            ss.m_cut = g.m_cut;
            ss.theta = p->theta;
        }
    }
    g.U0 = base + l.U0;
    g.U1 = base + l.U1;
    g.A = base + l.A;
    g.Bw = base + l.Bw;
    g.C = base + l.C;
    g.tw = base + l.tw;
    g.rate = base + l.rate;
    g.ones = reinterpret_cast<double*>(base + l.one);
    // the passes of ns_rhs with the built-in schedules (variant 0)
    NOALLOC_TRY(launch_pack(f64, uin, g.U0, g.L, g.K, s));
    const PassArgs a = pass_args(g, g.U0, g.U1, nullptr, 0.0, 0.0, 1.0, g.ones);
    for (int pass = 0; pass < NS_NPASS; ++pass) NOALLOC_TRY(launch_pass(g, pass, 0, a, s));
    NOALLOC_TRY(launch_unpack(f64, g.U1, rout, g.L, g.K, s));
    return NS_OK;
}

}  // extern "C"
