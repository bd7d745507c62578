/*
 * ns.h - C ABI of the MI355X spectral hyperviscosity Navier-Stokes library.
 *
 * The library advances the semi-discrete spectral hyperviscosity (SHV)
 * system for 3-D incompressible Navier-Stokes / Euler on the periodic box
 * [0, 2*pi]^3 (Rohner & Mishra, PASC '24, arXiv:2401.09843, Sec. 2.2,
 * eq. (2.1)) in Fourier space (Sec. 2.3, eq. (2.5)) with the third-order
 * strong-stability-preserving Runge-Kutta scheme of eq. (2.6).  Every step
 * of the computation runs in the library's own HIP kernels for gfx950.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid and transforms: x_j = 2*pi*j/N on each axis; the forward transform is
 * normalised, u-hat_k = N^-3 sum_x u(x) exp(-i k.x).  Index j along an axis
 * carries wavenumber j for j < N/2 and j - N otherwise.
 *
 * Public spectral layout ("R2C layout"): one sample's velocity spectrum is a
 * dense device array uhat[3][N][N][N/2+1] of interleaved complex numbers
 * (re, im) in the context's precision, component-major (u_x, u_y, u_z), then
 * k_z index, k_y index, k_x = 0..N/2 (x fastest).  It equals
 * numpy.fft.rfftn(u, axes=(-3,-2,-1), norm="forward") of the real field
 * u[3][z][y][x].  Modes outside the 2/3-rule cube |k_x|,|k_y|,|k_z| <= K,
 * K = floor((N-1)/3) (Algorithm 2, step 5; Sec. 2.2 for the cube), are
 * ignored on input and written as zero on output.  On the k_x = 0 plane the
 * real part of the real-space field is used, i.e. the plane is read as its
 * Hermitian part.
 *
 * Physical layout: u[3][N][N][N] real, (component, z, y, x), x fastest.
 *
 * Batches: a context holds nsamples samples with sizes n[i].  Array
 * arguments named "const* x" are HOST arrays of nsamples DEVICE pointers,
 * one per sample.  Samples of equal N run in the same kernel launches.
 *
 * Ownership: the caller owns every state, output, tape and adjoint buffer;
 * the context owns its plans, twiddle tables, workspaces and graphs and
 * frees them in ns_destroy.  A context must not be used from two host
 * threads at once.  All device work is enqueued on the stream given to
 * ns_init; calls return without synchronising unless stated.
 *
 * Errors: every call returns an ns_status and never aborts.  Bad arguments
 * give NS_ERR_ARG with nothing enqueued; the message is in ns_last_error.
 * A failed HIP call gives NS_ERR_HIP and makes the context sticky-failed:
 * later calls return NS_ERR_STATE.
 */
#ifndef NS_H
#define NS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_ctx ns_ctx;

typedef enum {
    NS_OK = 0,
    NS_ERR_ARG = 1,
    NS_ERR_UNSUPPORTED = 2,
    NS_ERR_OOM = 3,
    NS_ERR_HIP = 4,
    NS_ERR_STATE = 5,
    NS_ERR_NONFINITE = 6
} ns_status;

typedef enum { NS_F32 = 0, NS_F64 = 1 } ns_dtype;

/* flags */
#define NS_USE_GRAPH    1u  /* replay each RK3 step from a captured hipGraph */
#define NS_CHECK_FINITE 2u  /* ns_step checks the energy after the call */
#define NS_NO_TUNE      4u  /* skip the autotuner; use the built-in schedules */
#define NS_NO_FUSE      8u  /* stepping runs every stage as the plain five passes */
#define NS_FUSE        16u  /* stepping ends every stage in the fused pass: the forward
                               z pass also writes the inverse z transform of the new
                               state, and the next stage starts at its second pass.
                               With neither flag the autotuner times whole stages both
                               ways and keeps the faster form per grid size (with
                               NS_NO_TUNE: fused).  The two flags exclude each other. */
#define NS_PAD         32u  /* Algorithm 2 in its padded form: n[i] is the number of modes
                               per axis of the state, whose spectra use the n-point
                               half-spectrum layout, and the passes run on the grid of
                               3n/2 points (every product is then alias-free).  The state
                               holds |k_i| <= n/2 - 1: the Nyquist planes k_i = -n/2 are
                               ignored on input and written as zero.  Physical fields
                               (ns_forward, ns_inverse) live on the 3n/2 grid; eps and
                               m_cut defaults are taken at n. */
#define NS_GRAPH_CHAIN    64u  /* with NS_USE_GRAPH and several grid sizes: the captured
                                  step runs the size groups one after another on one
                                  stream */
#define NS_GRAPH_BRANCHES 128u /* ... or as concurrent graph branches.  With neither flag
                                  (and without NS_NO_TUNE) ns_init times both forms on
                                  seeded states and keeps the branches only if they win
                                  by more than 1 %; with NS_NO_TUNE: the chain.  The two
                                  flags exclude each other; results are bitwise the same
                                  in either form. */

/* Model and run parameters (eqs. (2.1)-(2.4)).
 *   eps    epsilon_N, the hyperviscosity amplitude; < 0 selects the default
 *          1e-3 * (32/N)^(2s-1) per sample (N: the sample's n[i]).
 *   s      hyperviscosity order: the damping symbol is |k|^{2s} (s >= 1).
 *   m_cut  m_N: Q-hat_k = 0 for |k| <= m_N; < 0 selects N/3 per sample.
 *   q_kind 0: Q-hat_k = 1 above m_N; 1: Q-hat_k = 1 - (m_N/|k|)^((2s-1)/theta)
 *          above m_N (the lower bound of eq. (2.3)).
 *   theta  the exponent parameter of eq. (2.4), used by q_kind 1.
 * The right-hand side is dissipative: F_k = ... - eps |k|^{2s} Q-hat_k u-hat_k. */
typedef struct {
    ns_dtype       dtype;
    int32_t        nsamples;   /* >= 1 */
    const int32_t* n;          /* host array [nsamples]: grid sizes N with compiled kernels
                                  (ns_supported_sizes: 8..1536, 2^a 3^b 5^c); with NS_PAD
                                  even mode counts n with 3n/2 supported */
    double         eps;
    double         s;
    double         m_cut;
    int32_t        q_kind;
    double         theta;
    uint32_t       flags;      /* NS_USE_GRAPH | NS_CHECK_FINITE | NS_NO_TUNE | NS_NO_FUSE | NS_FUSE | NS_PAD
                                  | NS_GRAPH_CHAIN | NS_GRAPH_BRANCHES */
    const char*    tune_cache; /* autotuner cache file (JSON) or NULL */
} ns_params;

/* Create a context on the current HIP device; hip_stream is a hipStream_t
 * (NULL = the default stream).  Allocates the workspaces; runs the
 * autotuner for each distinct N unless NS_NO_TUNE is set. */
ns_status ns_init(const ns_params* params, void* hip_stream, ns_ctx** out);

/* Free everything the context owns.  Accepts NULL. */
ns_status ns_destroy(ns_ctx* ctx);

/* Message of the last failure on ctx (context-owned, valid until the next
 * call); for a NULL ctx, the last ns_init failure of the calling thread. */
const char* ns_last_error(const ns_ctx* ctx);

/* Total bytes of device memory the context allocated. */
ns_status ns_workspace_bytes(const ns_ctx* ctx, size_t* bytes);

/* Supported grid sizes: writes up to cap values to sizes, count to *count. */
ns_status ns_supported_sizes(int32_t* sizes, int32_t cap, int32_t* count);

/* Initial data, eq. (2.1) third line with the divergence constraint:
 * uhat = T P F[u], from physical u[3][N][N][N] (R2C layout out).  In- and
 * output may not alias. */
ns_status ns_forward(ns_ctx* ctx, const void* const* u_phys, void* const* uhat);

/* Physical field u = F^-1[T uhat] (T = 2/3 truncation), real [3][N]^3. */
ns_status ns_inverse(ns_ctx* ctx, const void* const* uhat, void* const* u_phys);

/* T and the Leray projection (I - k k^T/|k|^2) in place (eq. (2.5)). */
ns_status ns_project(ns_ctx* ctx, void* const* uhat);

/* One evaluation of the right-hand side (Algorithm 2 with eq. (2.5)):
 *   rhs = T[ P(-i k . F[u (x) u]) - eps |k|^{2s} Q-hat u-hat ],
 * with u (x) u formed pointwise on the N^3 grid from u = F^-1[T uhat] and
 * its transform 2/3-truncated.  uhat_in and rhs_out may not alias. */
ns_status ns_rhs(ns_ctx* ctx, const void* const* uhat_in, void* const* rhs_out);

/* nsteps SSP-RK3 steps (eq. (2.6)) of fixed size dt[i] (host array
 * [nsamples], finite and > 0) in place on uhat.  nsteps >= 0.  With
 * NS_CHECK_FINITE, synchronises and returns NS_ERR_NONFINITE if a sample's
 * energy is not finite at the end. */
ns_status ns_step(ns_ctx* ctx, void* const* uhat_inout, const double* dt, int32_t nsteps);

/* Bytes of tape per sample that ns_step_taped writes for nsteps steps (the
 * largest over the context's grid sizes). */
ns_status ns_tape_bytes(const ns_ctx* ctx, int32_t nsteps, size_t* per_sample);

/* Bytes of one step of the tape of a sample of size n (as in params->n):
 * the step stride of that sample's tape, whose step k starts at
 * k * *bytes.  NS_ERR_ARG if the context holds no sample of size n. */
ns_status ns_tape_step_bytes(const ns_ctx* ctx, int32_t n, size_t* bytes);

/* As ns_step, and also records each step's three stage states into tape[i]
 * (opaque, ns_tape_bytes(nsteps) bytes per sample), for ns_adjoint_step. */
ns_status ns_step_taped(ns_ctx* ctx, void* const* uhat_inout, const double* dt, int32_t nsteps,
                        void* const* tape);

/* Discrete adjoint of one SSP-RK3 step (not in the paper: the transpose of
 * the Jacobian of the step in the inner product <a,b> = Re sum over the full
 * spectrum of conj(a_k) b_k).  lam (R2C layout) holds dJ/du^{n+1} on entry
 * and dJ/du^n on return.  The stage states come from tape_step[i] (one step
 * of a tape written by ns_step_taped, i.e. tape + step * per_step_bytes) or,
 * if tape_step is NULL, are recomputed from uhat_n (the step's input).
 * As for every entry point, modes of lam outside the 2/3 cube are ignored
 * (the step maps them to zero, so their adjoint is zero) and written as 0. */
ns_status ns_adjoint_step(ns_ctx* ctx, const void* const* uhat_n, const void* const* tape_step,
                          const double* dt, void* const* lam_inout);

/* nsteps adjoint steps backward through a whole tape written by
 * ns_step_taped(nsteps): lam holds dJ/du at the end of the taped steps on
 * entry and dJ/du at their start on return (steps nsteps-1 .. 0; lam stays
 * in the compact layout in between). */
ns_status ns_adjoint_steps(ns_ctx* ctx, const void* const* tape, int32_t nsteps, const double* dt,
                           void* const* lam_inout);

/* Energy spectrum (the energy-spectrum writer of Sec. 2.4):
 * E[i][kappa] = 1/2 sum over modes of the full spectrum with
 * round(|k|) = kappa of |u-hat_k|^2, kappa = 0..kbins-1, written as FP64
 * into the DEVICE array E_dev[nsamples][kbins].  Deterministic. */
ns_status ns_energy_spectrum(ns_ctx* ctx, const void* const* uhat, double* E_dev, int32_t kbins);

/* Enstrophy spectrum (the enstrophy-spectrum writer of Sec. 2.4):
 * Z[i][kappa] = 1/2 sum over modes of the full spectrum with
 * round(|k|) = kappa of |k x u-hat_k|^2 (the vorticity is i k x u-hat), same
 * shells, layout and determinism as ns_energy_spectrum. */
ns_status ns_enstrophy_spectrum(ns_ctx* ctx, const void* const* uhat, double* Z_dev, int32_t kbins);

/* Pointwise statistics of the empirical measure of Algorithm 1 (step 3)
 * over the samples of size n: with u_b = F^-1[T uhat_b] on the sample grid
 * (N = n, or 3n/2 with NS_PAD), mean = (1/B) sum_b u_b and var = (1/B)
 * sum_b (u_b - mean)^2, accumulated in FP64 in sample order (deterministic):
 * the group's samples go back to the grid in batched passes, then one
 * Welford pass per point.
 * uhat: host array [nsamples] as for every call (samples of other sizes are
 * not read); mean_dev and var_dev: distinct device arrays of doubles
 * [3][N][N][N], overwritten.  Uses the size group's workspaces. */
ns_status ns_moments(ns_ctx* ctx, const void* const* uhat, int32_t n, double* mean_dev, double* var_dev);

/* Longitudinal velocity structure functions of order p (the structure-
 * function writers of Sec. 2.4; reading: increments of each component along
 * its own axis, averaged over the three axes):
 *   S[i][l-1] = 1/3 sum_d mean_x |u_d(x + l h e_d) - u_d(x)|^p, l = 1..lmax,
 * for u = F^-1[T uhat_i] on the sample's grid (spacing h = 2 pi / N).
 * S_dev: device doubles [nsamples][lmax]; 1 <= lmax <= N/2 for every
 * sample, p > 0.  Deterministic; uses the group's workspaces. */
ns_status ns_structure_functions(ns_ctx* ctx, const void* const* uhat, int32_t lmax, double p, double* S_dev);

/* Distance between the 1-point marginals of two ensembles (the statistic of
 * the paper's convergence study, Sec. 6.1): for each velocity component and
 * grid point, the 1-D Wasserstein-1 distance W1 = integral |F_a - F_b| dt
 * between the empirical distributions of the na values of ensemble a and the
 * nb values of ensemble b (component by component, a reading of the paper's
 * vector-valued marginals).  a: device array [na][3][n][n][n], b:
 * [nb][3][n][n][n], physical fields of the context's real type (e.g. from
 * ns_inverse); w_dev: device doubles [3][n][n][n] (the pointwise distance,
 * overwritten); mean_dev: device doubles [3], the mean of w over the points
 * per component, or NULL.  na, nb >= 1, na + nb <= 20480; the values are
 * sorted per point in LDS, O((na + nb)^2) work per point.  Deterministic. */
ns_status ns_wasserstein1(ns_ctx* ctx, const void* a, int32_t na, const void* b, int32_t nb, int32_t n,
                          double* w_dev, double* mean_dev);

/* Allocation-free right-hand side, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the result of ns_rhs for one sample, without a context.
 *   params     as for ns_init with nsamples = 1 and n[0] the sample's size;
 *              dtype, eps, s, m_cut, q_kind, theta and NS_PAD are honoured,
 *              the other flags are ignored.  The passes use the built-in
 *              schedules (those of a context made with NS_NO_TUNE), so the
 *              output equals that context's ns_rhs bit for bit.
 *   uhat_in    device array, one spectrum in the R2C layout (as ns_rhs)
 *   rhs_out    device array of the same shape; may not alias uhat_in
 *   hip_stream hipStream_t (NULL = the default stream)
 * Workspaces: the compact states, the pass workspaces and the twiddle and
 * damping tables live in one static device array of
 * NS_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * until the process ends.  A grid N (3n/2 with NS_PAD) needs, with
 * K = floor((N-1)/3), M = 2K+1, Mx = K+1 and c the bytes of a complex number,
 * about c (6 M^2 Mx + 6 N M Mx + 9 N^2 Mx + N) bytes: N <= 96 in FP32 and
 * N <= 80 in FP64 fit.  Larger sizes give NS_ERR_ARG with nothing enqueued.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine.  When the table parameters (size, precision, eps, s, m_cut,
 * q_kind, theta) differ from the previous call's on that GPU, it uploads the
 * tables and synchronises the stream; otherwise it only enqueues kernels.
 * Every call on one GPU shares that GPU's array and leaves its contents for
 * the next: calls that overlap in time on one GPU (from several host threads
 * or on several streams) race and give undefined results.
 * Errors: NS_ERR_ARG / NS_ERR_UNSUPPORTED / NS_ERR_HIP; the message is
 * returned by ns_last_error(NULL) on the calling thread. */
#define NS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ns_status ns_rhs_noalloc(const ns_params* params, const void* uhat_in, void* rhs_out, void* hip_stream);

/* Synchronise the context's stream (convenience for callers without HIP). */
ns_status ns_sync(ns_ctx* ctx);

/* Pass profiler.  With enable != 0 every pass launch of ns_rhs / ns_step is
 * bracketed by HIP events on the context's stream (ns_step then launches
 * eagerly instead of replaying its graph).  ns_profile_read synchronises,
 * writes per pass p the summed device time in milliseconds ms[p] and the
 * number of launches count[p] since the last read, and resets them.
 * Passes: 0 = inverse z (I1), 1 = inverse y (I2), 2 = x (C2R, products,
 * R2C), 3 = forward y (F2), 4 = forward z + epilogue (F3).  Where the
 * stages are fused (NS_FUSE), ns_step runs pass 0 once per call and group,
 * and each pass 4 launch of a step also does the next stage's pass 0. */
#define NS_NPASS 5
ns_status ns_profile(ns_ctx* ctx, int32_t enable);
ns_status ns_profile_read(ns_ctx* ctx, double* ms, int64_t* count);

/* Schedule variants and the autotuner (the build's analogue of the per-
 * system FFT benchmark of Sec. 3.1).  Each pass of the samples of grid size
 * n has a list of compiled schedules (threads per line, radix order, tile
 * width, LDS exchange form, occupancy); all compute the same result.
 * Unless NS_NO_TUNE is set, ns_init times every variant on the context's
 * workspaces, keeps the fastest, and appends the choice to the tune_cache
 * file (one JSON object per line; read back when the key matches).
 * ns_set_variant overrides the choice (e.g. to test every variant; a pass 4
 * variant is used in the group's stage form); ns_tune_report writes the
 * choices and timings as JSON into buf, with the stage form ("fused") and
 * the stage timings on each pass-4 entry, and with several grid sizes the
 * graph launch form ("graph_form": "chain" or "branches", and its timings
 * "graph_ms", 0 when not timed) on those entries too (always
 * NUL-terminated; *needed receives the full length + 1). */
ns_status ns_variant_count(ns_ctx* ctx, int32_t n, int32_t pass, int32_t* count);
ns_status ns_set_variant(ns_ctx* ctx, int32_t n, int32_t pass, int32_t variant);
ns_status ns_tune_report(ns_ctx* ctx, char* buf, size_t len, size_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* NS_H */
