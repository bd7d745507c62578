/*
 * CPU oracle for the spectral hyperviscosity (SHV) Navier-Stokes right-hand
 * side and its SSP-RK3 time stepper (Rohner & Mishra, "Efficient Computation
 * of Large-Scale Statistical Solutions to Incompressible Fluid Flows",
 * PASC '24, arXiv:2401.09843).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
 * reference that the GPU path is compared against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code with the GPU library (no headers, tables or helpers).
 *
 * Conventions (the periodic box [0,2*pi]^3, integer wavenumbers):
 *   grid point x_j = 2*pi*j/N, j = 0..N-1 on each axis;
 *   forward  uhat_k = N^-3 sum_x u(x) exp(-i k.x);
 *   inverse  u(x)   = sum_k uhat_k exp(+i k.x);
 *   index j on an axis carries wavenumber j for j < N/2, j - N otherwise.
 * All spectra here are FULL complex N^3 arrays, layout [z][y][x], x fastest;
 * vector fields are [3][z][y][x] with components (u_x, u_y, u_z).
 * All arithmetic is IEEE double.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Model parameters.  eps = epsilon_N and s = hyperviscosity order of
 * eq. (2.1); m_cut = m_N of eq. (2.3); q_kind selects the multiplier Q-hat:
 * 0 = the step (Q=0 for |k| <= m_N, else 1), 1 = the lower bound of
 * eq. (2.3), 1-(m_N/|k|)^((2s-1)/theta), above m_N.  kcut is the dealiasing
 * cutoff K (keep |k_x|,|k_y|,|k_z| <= K); a negative value selects the
 * 2/3-rule default floor((N-1)/3). */
typedef struct {
    double eps;
    double s;
    double m_cut;
    int    q_kind;
    double theta;
    int    kcut;
} orc_params;

static int wavenumber(int j, int n) { return j < n / 2 ? j : j - n; }

static int default_kcut(int n) { return (n - 1) / 3; }

static int kcut_of(const orc_params *p, int n) { return p->kcut >= 0 ? p->kcut : default_kcut(n); }

/* The 2/3 truncation T of Algorithm 2, step 5 (cube in |k|_inf, Sec. 2.2). */
static int retained(int kx, int ky, int kz, int K)
{
    return abs(kx) <= K && abs(ky) <= K && abs(kz) <= K;
}

/* Hyperviscosity damping rate eps_N |k|^{2s} Q-hat_k of eqs. (2.1)-(2.3);
 * the right-hand side gets minus this rate times u-hat_k (dissipative sign). */
static double hyperviscous_rate(const orc_params *p, int kx, int ky, int kz)
{
    double k2 = (double)kx * kx + (double)ky * ky + (double)kz * kz;
    double kabs = sqrt(k2);
    double q;
    if (kabs <= p->m_cut) q = 0.0;
    else if (p->q_kind == 0) q = 1.0;
    else q = 1.0 - pow(p->m_cut / kabs, (2.0 * p->s - 1.0) / p->theta);
    return p->eps * pow(k2, p->s) * q;
}

/* ------------------------------------------------------------------------ */
/* 1-D DFT by plain recursive decimation in time over the smallest prime
 * factor; a prime length is summed directly.  tw[e] = exp(sign*2*pi*i*e/ntop)
 * is a table for the top-level length; a sub-length m uses tw[e*ntop/m].
 * out must not alias in; tmp holds at least n values.                      */
static int smallest_prime_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

static void dft_rec(int n, const cplx *in, long is, cplx *out, cplx *tmp, const cplx *tw, int ntop)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_prime_factor(n);
    int m = n / p;
    int step = ntop / n; /* exp(2 pi i e / n) = tw[e * step] */
    if (m == 1) {
        for (int k = 0; k < n; ++k) {
            cplx s = 0;
            for (int j = 0; j < n; ++j) s += in[j * is] * tw[(long)((j * k) % n) * step];
            out[k] = s;
        }
        return;
    }
    /* sub-transform r works on the inputs with index = r (mod p) */
    for (int r = 0; r < p; ++r) dft_rec(m, in + r * is, is * p, out + r * m, tmp, tw, ntop);
    for (int k = 0; k < n; ++k) {
        cplx s = 0;
        for (int r = 0; r < p; ++r) s += tw[(long)((r * k) % n) * step] * out[r * m + k % m];
        tmp[k] = s;
    }
    memcpy(out, tmp, sizeof(cplx) * n);
}

static cplx *twiddle_table(int n, int sign)
{
    cplx *tw = malloc(sizeof(cplx) * n);
    for (int e = 0; e < n; ++e) {
        double a = 2.0 * M_PI * (double)e / (double)n;
        tw[e] = cos(a) + sign * sin(a) * I;
    }
    return tw;
}

/* Unnormalised 1-D DFT: out[k] = sum_j in[j] exp(sign*2*pi*i*j*k/n). */
void orc_dft1(int n, const cplx *in, cplx *out, int sign)
{
    cplx *tw = twiddle_table(n, sign);
    cplx *tmp = malloc(sizeof(cplx) * n);
    dft_rec(n, in, 1, out, tmp, tw, n);
    free(tmp);
    free(tw);
}

/* Unnormalised 3-D DFT of an N^3 array in place, one axis at a time. */
void orc_fft3(int n, cplx *a, int sign)
{
    cplx *tw = twiddle_table(n, sign);
    long n2 = (long)n * n;
    for (int axis = 0; axis < 3; ++axis) {
        long stride = axis == 0 ? 1 : (axis == 1 ? n : n2);
#pragma omp parallel
        {
            cplx *line = malloc(sizeof(cplx) * n);
            cplx *res = malloc(sizeof(cplx) * n);
            cplx *tmp = malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
            for (long l = 0; l < n2; ++l) {
                /* line l: the two indices other than the transformed one */
                long a0 = l / n, a1 = l % n, base;
                if (axis == 0) base = a0 * n2 + a1 * n;      /* z, y fixed */
                else if (axis == 1) base = a0 * n2 + a1;     /* z, x fixed */
                else base = a0 * n + a1;                     /* y, x fixed */
                for (int j = 0; j < n; ++j) line[j] = a[base + j * stride];
                dft_rec(n, line, 1, res, tmp, tw, n);
                for (int j = 0; j < n; ++j) a[base + j * stride] = res[j];
            }
            free(line);
            free(res);
            free(tmp);
        }
    }
    free(tw);
}

/* The definition of the 3-D DFT summed term by term, O(N^6); for N <= 8. */
void orc_dft3_brute(int n, const cplx *in, cplx *out, int sign)
{
    for (int kz = 0; kz < n; ++kz)
        for (int ky = 0; ky < n; ++ky)
            for (int kx = 0; kx < n; ++kx) {
                cplx s = 0;
                for (int z = 0; z < n; ++z)
                    for (int y = 0; y < n; ++y)
                        for (int x = 0; x < n; ++x) {
                            long e = ((long)kz * z + (long)ky * y + (long)kx * x) % n;
                            double a = 2.0 * M_PI * (double)e / (double)n;
                            s += in[((long)z * n + y) * n + x] * (cos(a) + sign * sin(a) * I);
                        }
                out[((long)kz * n + ky) * n + kx] = s;
            }
}

/* Normalised forward transform of one scalar field: N^-3 * DFT(sign -1). */
static void forward3(int n, cplx *a)
{
    orc_fft3(n, a, -1);
    long n3 = (long)n * n * n;
    double sc = 1.0 / (double)n3;
    for (long i = 0; i < n3; ++i) a[i] *= sc;
}

static void inverse3(int n, cplx *a) { orc_fft3(n, a, +1); }

/* Zero every mode outside the truncation cube. */
static void truncate_field(int n, int K, cplx *a)
{
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x)
                if (!retained(wavenumber(x, n), wavenumber(y, n), wavenumber(z, n), K))
                    a[((long)z * n + y) * n + x] = 0;
}

/* Leray projection of one mode, (I - k k^T/|k|^2) v, eq. (2.5); k = 0 is
 * left unchanged (a constant field is divergence free). */
static void leray(int kx, int ky, int kz, cplx *v0, cplx *v1, cplx *v2)
{
    double k2 = (double)kx * kx + (double)ky * ky + (double)kz * kz;
    if (k2 == 0.0) return;
    cplx kv = kx * *v0 + ky * *v1 + kz * *v2;
    *v0 -= kx * kv / k2;
    *v1 -= ky * kv / k2;
    *v2 -= kz * kv / k2;
}

/* Initial projection T P (eq. (2.1), third line, plus the divergence-free
 * constraint) of a full spectrum [3][N^3], in place. */
void orc_project(int n, const orc_params *p, cplx *uh)
{
    int K = kcut_of(p, n);
    long n3 = (long)n * n * n;
    truncate_field(n, K, uh);
    truncate_field(n, K, uh + n3);
    truncate_field(n, K, uh + 2 * n3);
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long i = ((long)z * n + y) * n + x;
                leray(wavenumber(x, n), wavenumber(y, n), wavenumber(z, n), uh + i, uh + n3 + i, uh + 2 * n3 + i);
            }
}

/* Physical real field [3][N^3] -> full spectrum [3][N^3], normalised. */
void orc_forward(int n, const double *u, cplx *uh)
{
    long n3 = (long)n * n * n;
    for (long i = 0; i < 3 * n3; ++i) uh[i] = u[i];
    for (int c = 0; c < 3; ++c) forward3(n, uh + c * n3);
}

/* Full spectrum [ncomp][N^3] -> physical [ncomp][N^3]; returns the largest
 * |imaginary part| met (zero up to rounding for a Hermitian input). */
double orc_inverse(int n, int ncomp, const cplx *uh, double *u)
{
    long n3 = (long)n * n * n;
    cplx *w = malloc(sizeof(cplx) * n3);
    double maximag = 0.0;
    for (int c = 0; c < ncomp; ++c) {
        memcpy(w, uh + c * n3, sizeof(cplx) * n3);
        inverse3(n, w);
        for (long i = 0; i < n3; ++i) {
            u[c * n3 + i] = creal(w[i]);
            if (fabs(cimag(w[i])) > maximag) maximag = fabs(cimag(w[i]));
        }
    }
    free(w);
    return maximag;
}

/* The six upper-triangular components of the symmetric tensor u (x) u. */
static const int TRI_I[6] = {0, 0, 0, 1, 1, 2};
static const int TRI_J[6] = {0, 1, 2, 1, 2, 2};

static int tri_index(int i, int j)
{
    if (i > j) { int t = i; i = j; j = t; }
    for (int q = 0; q < 6; ++q)
        if (TRI_I[q] == i && TRI_J[q] == j) return q;
    return -1;
}

/* Right-hand side F(u-hat) of the semi-discrete SHV system, Algorithm 2 with
 * eq. (2.5):
 *   u = F^-1[T u-hat];  B_ij = u_i u_j (i <= j);  B-hat = T F[B];
 *   b_i = -i sum_j k_j B-hat_ij;  c = (I - k k^T/|k|^2) b  (c_0 = 0);
 *   F = T[ c - eps |k|^{2s} Q(|k|) u-hat ].
 * uh and out are full spectra [3][N^3]; they may not alias.  Returns the
 * largest imaginary residue of the inverse transforms. */
double orc_rhs(int n, const orc_params *p, const cplx *uh, cplx *out)
{
    int K = kcut_of(p, n);
    long n3 = (long)n * n * n;
    cplx *ut = malloc(sizeof(cplx) * 3 * n3);
    double *u = malloc(sizeof(double) * 3 * n3);
    cplx *B = malloc(sizeof(cplx) * 6 * n3);
    memcpy(ut, uh, sizeof(cplx) * 3 * n3);
    for (int c = 0; c < 3; ++c) truncate_field(n, K, ut + c * n3);
    double maximag = orc_inverse(n, 3, ut, u);
    for (int q = 0; q < 6; ++q) {
        const double *ui = u + TRI_I[q] * n3, *uj = u + TRI_J[q] * n3;
        for (long x = 0; x < n3; ++x) B[q * n3 + x] = ui[x] * uj[x];
        forward3(n, B + q * n3);
        truncate_field(n, K, B + q * n3);
    }
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long id = ((long)z * n + y) * n + x;
                int k[3] = {wavenumber(x, n), wavenumber(y, n), wavenumber(z, n)};
                if (!retained(k[0], k[1], k[2], K)) {
                    out[id] = out[n3 + id] = out[2 * n3 + id] = 0;
                    continue;
                }
                cplx b[3];
                for (int i = 0; i < 3; ++i) {
                    cplx s = 0;
                    for (int j = 0; j < 3; ++j) s += k[j] * B[tri_index(i, j) * n3 + id];
                    b[i] = -I * s;
                }
                leray(k[0], k[1], k[2], &b[0], &b[1], &b[2]);
                double rate = hyperviscous_rate(p, k[0], k[1], k[2]);
                for (int i = 0; i < 3; ++i) out[i * n3 + id] = b[i] - rate * ut[i * n3 + id];
            }
    free(ut);
    free(u);
    free(B);
    return maximag;
}

/* SSP-RK3 of eq. (2.6), Shu-Osher form, nsteps steps of fixed dt, in place
 * on a full spectrum [3][N^3]. */
void orc_ssprk3(int n, const orc_params *p, cplx *uh, double dt, int nsteps)
{
    long m = 3L * n * n * n;
    cplx *u1 = malloc(sizeof(cplx) * m);
    cplx *u2 = malloc(sizeof(cplx) * m);
    cplx *f = malloc(sizeof(cplx) * m);
    for (int step = 0; step < nsteps; ++step) {
        orc_rhs(n, p, uh, f);
        for (long i = 0; i < m; ++i) u1[i] = uh[i] + dt * f[i];
        orc_rhs(n, p, u1, f);
        for (long i = 0; i < m; ++i) u2[i] = 0.75 * uh[i] + 0.25 * u1[i] + 0.25 * dt * f[i];
        orc_rhs(n, p, u2, f);
        for (long i = 0; i < m; ++i) uh[i] = uh[i] / 3.0 + (2.0 / 3.0) * u2[i] + (2.0 / 3.0) * dt * f[i];
    }
    free(u1);
    free(u2);
    free(f);
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint.  The paper states no adjoint; this is the transpose of
 * the Jacobian of orc_rhs in the inner product <a,b> = Re sum_k conj(a_k) b_k
 * over the full spectrum (N^-3 times the grid inner product by Parseval):
 *   mu = P T lambda;  S_ij = (d_i mu_j + d_j mu_i)/2  (S-hat = i/2 (k_i mu_j + k_j mu_i));
 *   a_i = 2 sum_j S_ij u_j   (grid product with u = F^-1[T u-hat]);
 *   F'(u)^T lambda = T F[a] - eps |k|^{2s} Q T lambda.
 * Derived by integrating the divergence form of the nonlinear term by parts:
 * <mu, -i k_j F[u_i v_j + v_i u_j]> = N^-3 sum_x v . a for every v in T. */
void orc_rhs_vjp(int n, const orc_params *p, const cplx *uh, const cplx *lam, cplx *out)
{
    int K = kcut_of(p, n);
    long n3 = (long)n * n * n;
    cplx *ut = malloc(sizeof(cplx) * 3 * n3);
    cplx *mu = malloc(sizeof(cplx) * 3 * n3);
    cplx *S = malloc(sizeof(cplx) * 6 * n3);
    double *u = malloc(sizeof(double) * 3 * n3);
    double *s = malloc(sizeof(double) * 6 * n3);
    memcpy(ut, uh, sizeof(cplx) * 3 * n3);
    memcpy(mu, lam, sizeof(cplx) * 3 * n3);
    for (int c = 0; c < 3; ++c) {
        truncate_field(n, K, ut + c * n3);
        truncate_field(n, K, mu + c * n3);
    }
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long i = ((long)z * n + y) * n + x;
                leray(wavenumber(x, n), wavenumber(y, n), wavenumber(z, n), mu + i, mu + n3 + i, mu + 2 * n3 + i);
            }
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long id = ((long)z * n + y) * n + x;
                int k[3] = {wavenumber(x, n), wavenumber(y, n), wavenumber(z, n)};
                for (int q = 0; q < 6; ++q) {
                    int i = TRI_I[q], j = TRI_J[q];
                    S[q * n3 + id] = 0.5 * I * (k[i] * mu[j * n3 + id] + k[j] * mu[i * n3 + id]);
                }
            }
    orc_inverse(n, 3, ut, u);
    orc_inverse(n, 6, S, s);
    cplx *a = S; /* reuse: the first three fields of S hold a */
    for (long x = 0; x < n3; ++x) {
        double av[3];
        for (int i = 0; i < 3; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) acc += s[tri_index(i, j) * n3 + x] * u[j * n3 + x];
            av[i] = 2.0 * acc;
        }
        for (int i = 0; i < 3; ++i) a[i * n3 + x] = av[i];
    }
    for (int c = 0; c < 3; ++c) {
        forward3(n, a + c * n3);
        truncate_field(n, K, a + c * n3);
    }
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long id = ((long)z * n + y) * n + x;
                int kx = wavenumber(x, n), ky = wavenumber(y, n), kz = wavenumber(z, n);
                if (!retained(kx, ky, kz, K)) {
                    out[id] = out[n3 + id] = out[2 * n3 + id] = 0;
                    continue;
                }
                double rate = hyperviscous_rate(p, kx, ky, kz);
                for (int i = 0; i < 3; ++i) out[i * n3 + id] = a[i * n3 + id] - rate * lam[i * n3 + id];
            }
    free(ut);
    free(mu);
    free(S);
    free(u);
    free(s);
}

/* Adjoint of one SSP-RK3 step: lam holds dJ/du^{n+1} on entry and dJ/du^n on
 * return; uh is the step's input state u^n (the stages are recomputed).
 * Transposes u1 = u + dt F(u), u2 = 3/4 u + 1/4 u1 + 1/4 dt F(u1),
 * u3 = 1/3 u + 2/3 u2 + 2/3 dt F(u2) stage by stage in reverse. */
void orc_adjoint_step(int n, const orc_params *p, const cplx *uh, double dt, cplx *lam)
{
    long m = 3L * n * n * n;
    cplx *u1 = malloc(sizeof(cplx) * m);
    cplx *u2 = malloc(sizeof(cplx) * m);
    cplx *f = malloc(sizeof(cplx) * m);
    cplx *l2 = malloc(sizeof(cplx) * m);
    cplx *l1 = malloc(sizeof(cplx) * m);
    orc_rhs(n, p, uh, f);
    for (long i = 0; i < m; ++i) u1[i] = uh[i] + dt * f[i];
    orc_rhs(n, p, u1, f);
    for (long i = 0; i < m; ++i) u2[i] = 0.75 * uh[i] + 0.25 * u1[i] + 0.25 * dt * f[i];
    /* lambda_2 = 2/3 lambda_3 + 2/3 dt F'(u2)^T lambda_3 */
    orc_rhs_vjp(n, p, u2, lam, f);
    for (long i = 0; i < m; ++i) l2[i] = (2.0 / 3.0) * lam[i] + (2.0 / 3.0) * dt * f[i];
    /* lambda_1 = 1/4 lambda_2 + 1/4 dt F'(u1)^T lambda_2 */
    orc_rhs_vjp(n, p, u1, l2, f);
    for (long i = 0; i < m; ++i) l1[i] = 0.25 * l2[i] + 0.25 * dt * f[i];
    /* lambda_n = 1/3 lambda_3 + 3/4 lambda_2 + lambda_1 + dt F'(u)^T lambda_1 */
    orc_rhs_vjp(n, p, uh, l1, f);
    for (long i = 0; i < m; ++i) lam[i] = lam[i] / 3.0 + 0.75 * l2[i] + l1[i] + dt * f[i];
    free(u1);
    free(u2);
    free(f);
    free(l2);
    free(l1);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics. */

/* Energy spectrum (the in-situ energy-spectrum writer of Sec. 2.4):
 * E[kappa] = 1/2 sum over k with round(|k|) = kappa of |u-hat_k|^2, over the
 * full spectrum; shells beyond nbins-1 are dropped. */
void orc_energy_spectrum(int n, const cplx *uh, double *E, int nbins)
{
    long n3 = (long)n * n * n;
    for (int b = 0; b < nbins; ++b) E[b] = 0.0;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long id = ((long)z * n + y) * n + x;
                int kx = wavenumber(x, n), ky = wavenumber(y, n), kz = wavenumber(z, n);
                int kappa = (int)lround(sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz));
                if (kappa >= nbins) continue;
                double e = 0.0;
                for (int c = 0; c < 3; ++c) {
                    cplx v = uh[c * n3 + id];
                    e += creal(v) * creal(v) + cimag(v) * cimag(v);
                }
                E[kappa] += 0.5 * e;
            }
}

/* Relative size of the divergent part: ||(I-P) u-hat|| / ||u-hat||. */
double orc_div_rel(int n, const cplx *uh)
{
    long n3 = (long)n * n * n;
    double num = 0.0, den = 0.0;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                long id = ((long)z * n + y) * n + x;
                int kx = wavenumber(x, n), ky = wavenumber(y, n), kz = wavenumber(z, n);
                double k2 = (double)kx * kx + (double)ky * ky + (double)kz * kz;
                cplx v[3] = {uh[id], uh[n3 + id], uh[2 * n3 + id]};
                for (int c = 0; c < 3; ++c) den += creal(v[c] * conj(v[c]));
                if (k2 == 0.0) continue;
                cplx kv = kx * v[0] + ky * v[1] + kz * v[2];
                num += creal(kv * conj(kv)) / k2;
            }
    return den > 0.0 ? sqrt(num / den) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of a field with a sparse spectrum, at chosen output modes,
 * from the Galerkin definition (valid at any N because 3K < N):
 *   b_i(k) = -i sum_j k_j sum_{p+q=k} u_i(p) u_j(q)   (p, q over the inputs),
 *   c = (I - k k^T/|k|^2) b,  F(k) = c - eps |k|^{2s} Q u(k).
 * kin[3*nin] / uin[3*nin] are the input modes (full spectrum: both k and -k
 * of a real field must be listed) and their three components; kout[3*nout]
 * the output modes (all inside T); out[3*nout] receives F. */
void orc_rhs_sparse(const orc_params *p, int nin, const int *kin, const cplx *uin, int nout, const int *kout,
                    cplx *out)
{
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < nout; ++o) {
        const int *k = kout + 3 * o;
        cplx b[3] = {0, 0, 0};
        cplx uk[3] = {0, 0, 0};
        for (int a = 0; a < nin; ++a) {
            const int *pa = kin + 3 * a;
            if (pa[0] == k[0] && pa[1] == k[1] && pa[2] == k[2])
                for (int i = 0; i < 3; ++i) uk[i] = uin[3 * a + i];
            for (int c = 0; c < nin; ++c) {
                const int *qc = kin + 3 * c;
                if (pa[0] + qc[0] != k[0] || pa[1] + qc[1] != k[1] || pa[2] + qc[2] != k[2]) continue;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) b[i] += k[j] * uin[3 * a + i] * uin[3 * c + j];
            }
        }
        for (int i = 0; i < 3; ++i) b[i] *= -I;
        leray(k[0], k[1], k[2], &b[0], &b[1], &b[2]);
        double rate = hyperviscous_rate(p, k[0], k[1], k[2]);
        for (int i = 0; i < 3; ++i) out[3 * o + i] = b[i] - rate * uk[i];
    }
}

/* Threads the oracle's parallel loops use (for reporting its timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
