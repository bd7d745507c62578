// Size-independent kernels: conversion between the public half-spectrum
// (R2C) layout and the compact retained-mode layout, the in-place
// truncation + Leray projection (eq. (2.5)), and the energy spectrum
// (the energy-spectrum writer of Sec. 2.4).
#include <cmath>

#include "args.hpp"
#include "fft_engine.hpp"
#include "misc_kernels.hpp"

namespace ns {

namespace {

__device__ __forceinline__ int full_index(int j, int K, int M, int N) { return j <= K ? j : j - M + N; }

// R2C [3][N][N][N/2+1] -> compact (the column-blocked layout of args.hpp)
template <typename R>
__global__ void k_pack(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out, int N, int K)
{
    const int M = 2 * K + 1, Mx = K + 1, Nh = N / 2 + 1;
    const long long total = 3LL * M * M * Mx;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    long long r = idx;
    const int kx = (int)(r % Mx);
    r /= Mx;
    const int jy = (int)(r % M);
    r /= M;
    const int jz = (int)(r % M);
    const int c = (int)(r / M);
    const int nz = full_index(jz, K, M, N), ny = full_index(jy, K, M, N);
    out[compact_off(sizeof(cpx<R>), 3, M, c, jz, (long long)jy * Mx + kx)] = in[(((long long)c * N + nz) * N + ny) * Nh + kx];
}

// compact -> R2C, zero outside the retained cube
template <typename R>
__global__ void k_unpack(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out, int N, int K)
{
    const int M = 2 * K + 1, Mx = K + 1, Nh = N / 2 + 1;
    const long long total = 3LL * N * N * Nh;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    long long r = idx;
    const int kx = (int)(r % Nh);
    r /= Nh;
    const int ny = (int)(r % N);
    r /= N;
    const int nz = (int)(r % N);
    const int c = (int)(r / N);
    const int jy = ny <= K ? ny : (ny >= N - K ? ny - N + M : -1);
    const int jz = nz <= K ? nz : (nz >= N - K ? nz - N + M : -1);
    cpx<R> v = {0, 0};
    if (kx <= K && jy >= 0 && jz >= 0) v = in[compact_off(sizeof(cpx<R>), 3, M, c, jz, (long long)jy * Mx + kx)];
    out[idx] = v;
}

// in place on R2C: zero outside the cube, Leray projection inside
template <typename R>
__global__ void k_project(cpx<R>* u, int N, int K)
{
    const int Nh = N / 2 + 1;
    const long long plane = (long long)N * N * Nh;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= plane) return;
    const int kxi = (int)(idx % Nh);
    const int ny = (int)((idx / Nh) % N);
    const int nz = (int)(idx / ((long long)Nh * N));
    const int kyi = ny < N / 2 ? ny : ny - N, kzi = nz < N / 2 ? nz : nz - N;
    cpx<R> v0 = u[idx], v1 = u[plane + idx], v2 = u[2 * plane + idx];
    if (kxi > K || kyi > K || -kyi > K || kzi > K || -kzi > K) {
        v0 = v1 = v2 = {0, 0};
    } else {
        const int k2 = kxi * kxi + kyi * kyi + kzi * kzi;
        if (k2 > 0) {
            const R kx = (R)kxi, ky = (R)kyi, kz = (R)kzi, inv = (R)1 / (R)k2;
            const R bx = (kx * v0.x + ky * v1.x + kz * v2.x) * inv;
            const R by = (kx * v0.y + ky * v1.y + kz * v2.y) * inv;
            v0.x -= kx * bx;
            v0.y -= kx * by;
            v1.x -= ky * bx;
            v1.y -= ky * by;
            v2.x -= kz * bx;
            v2.y -= kz * by;
        }
    }
    u[idx] = v0;
    u[plane + idx] = v1;
    u[2 * plane + idx] = v2;
}

__device__ __forceinline__ long long isqrt_ll(long long v)
{
    if (v <= 0) return 0;
    long long r = (long long)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// One block per shell kappa: E[kappa] = 1/2 sum |u_k|^2 over retained modes
// with kappa^2 - kappa < |k|^2 <= kappa^2 + kappa (i.e. round(|k|) = kappa;
// shell 0 is |k| = 0 alone),
// weight 2 for k_x > 0 (the mirrored half).  Each thread walks a fixed set
// of (k_z, k_y) rows in order and the block reduces in a fixed tree, so the
// result is bitwise reproducible.
constexpr int SPEC_THREADS = 256;

// KIND 0: energy, e = |u-hat_k|^2; KIND 1: enstrophy, e = |k x u-hat_k|^2
// (the vorticity omega-hat = i k x u-hat).
template <typename R, int KIND>
__global__ void __launch_bounds__(SPEC_THREADS) k_spectrum(const cpx<R>* __restrict__ u, double* E, int N, int K,
                                                           int kbins)
{
    __shared__ double red[SPEC_THREADS];
    const int kappa = blockIdx.x;
    const int Nh = N / 2 + 1, M = 2 * K + 1;
    const long long plane = (long long)N * N * Nh;
    // |k|^2 > kappa^2 - kappa, except that shell 0 starts at |k| = 0
    const long long lo2 = kappa == 0 ? -1 : (long long)kappa * kappa - kappa;
    const long long hi2 = (long long)kappa * kappa + kappa;
    double acc = 0.0;
    for (int r = threadIdx.x; r < M * M; r += SPEC_THREADS) {
        const int jz = r / M, jy = r % M;
        const int kz = jz <= K ? jz : jz - M, ky = jy <= K ? jy : jy - M;
        const long long q = (long long)kz * kz + (long long)ky * ky;
        const long long B = hi2 - q;
        if (B < 0) continue;
        const long long A = lo2 - q;
        const int lo = A < 0 ? 0 : (int)isqrt_ll(A) + 1;
        int hi = (int)isqrt_ll(B);
        if (hi > K) hi = K;
        const int nz = kz < 0 ? kz + N : kz, ny = ky < 0 ? ky + N : ky;
        const long long base = ((long long)nz * N + ny) * Nh;
        for (int kx = lo; kx <= hi; ++kx) {
            double e = 0.0;
            if constexpr (KIND == 0) {
                for (int c = 0; c < 3; ++c) {
                    const cpx<R> v = u[c * plane + base + kx];
                    e += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
                }
            } else {
                const cpx<R> a = u[base + kx], b = u[plane + base + kx], w = u[2 * plane + base + kx];
                const double k0 = kx, k1 = ky, k2 = kz;
                // (k x u)_x = ky w - kz v, (k x u)_y = kz u - kx w, (k x u)_z = kx v - ky u
                const double cxr = k1 * w.x - k2 * b.x, cxi = k1 * w.y - k2 * b.y;
                const double cyr = k2 * a.x - k0 * w.x, cyi = k2 * a.y - k0 * w.y;
                const double czr = k0 * b.x - k1 * a.x, czi = k0 * b.y - k1 * a.y;
                e = cxr * cxr + cxi * cxi + cyr * cyr + cyi * cyi + czr * czr + czi * czi;
            }
            acc += (kx == 0 ? 0.5 : 1.0) * e;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = SPEC_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && kappa < kbins) E[kappa] = red[0];
}

__global__ void k_fill(double* p, double v, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// uniform values in [-1, 1) from a counter-based integer hash of the index
// (SplitMix64 finaliser); used to give the autotuner realistic operands
template <typename R>
__global__ void k_fill_random(R* p, long long n, unsigned long long seed)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    p[i] = (R)((double)(z >> 11) * (1.0 / 4503599627370496.0) - 1.0);
}

inline unsigned nblocks(long long total, int threads) { return (unsigned)((total + threads - 1) / threads); }

}  // namespace

hipError_t launch_pack(bool f64, const void* in, void* out, int N, int K, hipStream_t s)
{
    const int M = 2 * K + 1;
    const long long total = 3LL * M * M * (K + 1);
    if (f64) hipLaunchKernelGGL(k_pack<double>, dim3(nblocks(total, 256)), dim3(256), 0, s, (const cpx<double>*)in, (cpx<double>*)out, N, K);
    else hipLaunchKernelGGL(k_pack<float>, dim3(nblocks(total, 256)), dim3(256), 0, s, (const cpx<float>*)in, (cpx<float>*)out, N, K);
    return hipGetLastError();
}

hipError_t launch_unpack(bool f64, const void* in, void* out, int N, int K, hipStream_t s)
{
    const long long total = 3LL * N * N * (N / 2 + 1);
    if (f64) hipLaunchKernelGGL(k_unpack<double>, dim3(nblocks(total, 256)), dim3(256), 0, s, (const cpx<double>*)in, (cpx<double>*)out, N, K);
    else hipLaunchKernelGGL(k_unpack<float>, dim3(nblocks(total, 256)), dim3(256), 0, s, (const cpx<float>*)in, (cpx<float>*)out, N, K);
    return hipGetLastError();
}

hipError_t launch_project(bool f64, void* u, int N, int K, hipStream_t s)
{
    const long long total = (long long)N * N * (N / 2 + 1);
    if (f64) hipLaunchKernelGGL(k_project<double>, dim3(nblocks(total, 256)), dim3(256), 0, s, (cpx<double>*)u, N, K);
    else hipLaunchKernelGGL(k_project<float>, dim3(nblocks(total, 256)), dim3(256), 0, s, (cpx<float>*)u, N, K);
    return hipGetLastError();
}

hipError_t launch_spectrum(bool f64, const void* u, double* E, int N, int K, int kbins, hipStream_t s, int kind)
{
    if (kbins <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(kbins, 256)), dim3(256), 0, s, E, 0.0, kbins);
    // shells beyond round(sqrt(3) K) are empty
    int kmax = (int)ceil(sqrt(3.0) * K) + 1;
    int nb = kbins < kmax ? kbins : kmax;
    if (f64 && kind == 0) hipLaunchKernelGGL((k_spectrum<double, 0>), dim3(nb), dim3(SPEC_THREADS), 0, s, (const cpx<double>*)u, E, N, K, kbins);
    else if (f64) hipLaunchKernelGGL((k_spectrum<double, 1>), dim3(nb), dim3(SPEC_THREADS), 0, s, (const cpx<double>*)u, E, N, K, kbins);
    else if (kind == 0) hipLaunchKernelGGL((k_spectrum<float, 0>), dim3(nb), dim3(SPEC_THREADS), 0, s, (const cpx<float>*)u, E, N, K, kbins);
    else hipLaunchKernelGGL((k_spectrum<float, 1>), dim3(nb), dim3(SPEC_THREADS), 0, s, (const cpx<float>*)u, E, N, K, kbins);
    return hipGetLastError();
}

// Pointwise mean and variance (1/B) over B samples x[b * n + i]: a Welford
// update per sample in sample order (d = v - mean; mean += d / k;
// m2 += d (v - mean)), in FP64, so the result is deterministic.
template <typename R>
__global__ void k_moments(const R* __restrict__ x, int B, long long n, double* __restrict__ mean,
                          double* __restrict__ var)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double mu = 0.0, m2 = 0.0;
    for (int b = 0; b < B; ++b) {
        const double v = (double)x[(long long)b * n + i];
        const double d = v - mu;
        mu += d / (double)(b + 1);
        m2 += d * (v - mu);
    }
    mean[i] = mu;
    var[i] = m2 / (double)B;
}

hipError_t launch_moments(bool f64, const void* x, int B, long long n, double* mean, double* var, hipStream_t s)
{
    if (n <= 0 || B <= 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_moments<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, (const double*)x, B, n, mean, var);
    else hipLaunchKernelGGL(k_moments<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, (const float*)x, B, n, mean, var);
    return hipGetLastError();
}

// 1-D Wasserstein-1 distance between the empirical distributions of
// a[s * npts + i] (s < na) and b[s * npts + i] (s < nb) at every position i:
// each thread sorts its two sample sets into its own LDS strip (insertion
// sort), then walks the merged order adding |F_a - F_b| times the gap to the
// next value (F = fraction of samples consumed so far).
template <typename R>
__global__ void k_w1(const R* __restrict__ a, int na, const R* __restrict__ b, int nb, long long npts,
                     double* __restrict__ w)
{
    extern __shared__ double strip[];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    double* sa = strip + (long long)threadIdx.x * (na + nb);
    double* sb = sa + na;
    for (int s = 0; s < na; ++s) {
        const double v = (double)a[(long long)s * npts + i];
        int j = s;
        while (j > 0 && sa[j - 1] > v) { sa[j] = sa[j - 1]; --j; }
        sa[j] = v;
    }
    for (int s = 0; s < nb; ++s) {
        const double v = (double)b[(long long)s * npts + i];
        int j = s;
        while (j > 0 && sb[j - 1] > v) { sb[j] = sb[j - 1]; --j; }
        sb[j] = v;
    }
    int ia = 0, ib = 0;
    double prev = sa[0] < sb[0] ? sa[0] : sb[0], acc = 0.0;
    while (ia < na || ib < nb) {
        const bool from_a = ib >= nb || (ia < na && sa[ia] <= sb[ib]);
        const double v = from_a ? sa[ia] : sb[ib];
        acc += fabs((double)ia / na - (double)ib / nb) * (v - prev);
        if (from_a) ++ia;
        else ++ib;
        prev = v;
    }
    w[i] = acc;
}

// out[c] = mean of x[c * per .. (c + 1) * per) for c < ncomp: one block per
// component, fixed-order strided sums and tree (deterministic).
__global__ void __launch_bounds__(256) k_block_mean(const double* __restrict__ x, long long per, double* out)
{
    __shared__ double red[256];
    const double* p = x + (long long)blockIdx.x * per;
    double acc = 0.0;
    for (long long j = threadIdx.x; j < per; j += 256) acc += p[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] / (double)per;
}

hipError_t launch_w1(bool f64, const void* a, int na, const void* b, int nb, long long npts, int ncomp, double* w,
                     double* mean, hipStream_t s)
{
    if (npts <= 0) return hipSuccess;
    // threads per block so that their strips fit in 160 KiB of LDS
    const size_t per_thread = sizeof(double) * (size_t)(na + nb);
    int threads = 64;
    while (threads > 1 && per_thread * threads > 163840) threads /= 2;
    if (per_thread * threads > 163840) return hipErrorInvalidValue;
    const size_t lds = per_thread * threads;
    static bool attr32 = false, attr64 = false;
    if (lds > 65536) {
        bool& done = f64 ? attr64 : attr32;
        if (!done) {
            const void* fn = f64 ? reinterpret_cast<const void*>(k_w1<double>) : reinterpret_cast<const void*>(k_w1<float>);
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    if (f64) hipLaunchKernelGGL(k_w1<double>, dim3(nblocks(npts, threads)), dim3(threads), lds, s, (const double*)a, na, (const double*)b, nb, npts, w);
    else hipLaunchKernelGGL(k_w1<float>, dim3(nblocks(npts, threads)), dim3(threads), lds, s, (const float*)a, na, (const float*)b, nb, npts, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !mean) return e;
    hipLaunchKernelGGL(k_block_mean, dim3(ncomp), dim3(256), 0, s, w, npts / ncomp, mean);
    return hipGetLastError();
}

// Longitudinal structure functions of B physical fields u [B][3][N][N][N]
// (x fastest): for shift l = blockIdx.y + 1 and sample b = blockIdx.z, block
// x sums |u_d(x + l e_d) - u_d(x)|^p over its strided share of the points
// and the three axes into part[(b lmax + l - 1) nblk + x]; k_sfun_final adds
// the nblk partial sums of each (b, l) in order.  Both orders are fixed, so
// the result is deterministic.  IP > 0: the integer power p = IP by
// multiplication; IP = 0: pow.
template <int IP>
__device__ __forceinline__ double abs_pow(double d, double p)
{
    if constexpr (IP == 0) {
        return pow(fabs(d), p);
    } else {
        const double a = fabs(d);
        double r = a;
#pragma unroll
        for (int k = 1; k < IP; ++k) r *= a;
        return r;
    }
}

template <typename R, int IP>
__global__ void __launch_bounds__(256) k_sfun(const R* __restrict__ u, int N, double p, double* part)
{
    __shared__ double red[256];
    const int l = blockIdx.y + 1;
    const long long n3 = (long long)N * N * N, plane = (long long)N * N;
    const R* ub = u + (long long)blockIdx.z * 3 * n3;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n3; i += (long long)gridDim.x * 256) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / plane);
        const long long ix = i - x + (x + l) % N;
        const long long iy = i + (long long)(((y + l) % N) - y) * N;
        const long long iz = i + (long long)(((z + l) % N) - z) * plane;
        acc += abs_pow<IP>((double)ub[ix] - (double)ub[i], p);
        acc += abs_pow<IP>((double)ub[n3 + iy] - (double)ub[n3 + i], p);
        acc += abs_pow<IP>((double)ub[2 * n3 + iz] - (double)ub[2 * n3 + i], p);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_sfun_final(const double* __restrict__ part, int nblk, int lmax, double scale, double* S)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= lmax) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(long long)l * nblk + b];
    S[l] = acc * scale;
}

int sfun_blocks(int N)
{
    const long long n3 = (long long)N * N * N;
    const long long b = (n3 + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

template <typename R>
static void sfun_dispatch(const R* u, int N, int lmax, int B, double p, double* part, hipStream_t s)
{
    const dim3 grid(sfun_blocks(N), lmax, B);
    // the range is checked before the conversion, which is undefined for |p| beyond int
    const int ip = (p >= 1 && p <= 6 && p == std::floor(p)) ? (int)p : 0;
    switch (ip) {
        case 1: hipLaunchKernelGGL((k_sfun<R, 1>), grid, dim3(256), 0, s, u, N, p, part); break;
        case 2: hipLaunchKernelGGL((k_sfun<R, 2>), grid, dim3(256), 0, s, u, N, p, part); break;
        case 3: hipLaunchKernelGGL((k_sfun<R, 3>), grid, dim3(256), 0, s, u, N, p, part); break;
        case 4: hipLaunchKernelGGL((k_sfun<R, 4>), grid, dim3(256), 0, s, u, N, p, part); break;
        case 5: hipLaunchKernelGGL((k_sfun<R, 5>), grid, dim3(256), 0, s, u, N, p, part); break;
        case 6: hipLaunchKernelGGL((k_sfun<R, 6>), grid, dim3(256), 0, s, u, N, p, part); break;
        default: hipLaunchKernelGGL((k_sfun<R, 0>), grid, dim3(256), 0, s, u, N, p, part); break;
    }
}

hipError_t launch_sfun(bool f64, const void* u, int N, int lmax, int B, double p, double* part, hipStream_t s)
{
    if (lmax <= 0 || B <= 0) return hipSuccess;
    if (f64) sfun_dispatch((const double*)u, N, lmax, B, p, part, s);
    else sfun_dispatch((const float*)u, N, lmax, B, p, part, s);
    return hipGetLastError();
}

hipError_t launch_sfun_final(const double* part, int N, int lmax, double* S, hipStream_t s)
{
    hipLaunchKernelGGL(k_sfun_final, dim3((lmax + 63) / 64), dim3(64), 0, s, part, sfun_blocks(N), lmax,
                       1.0 / (3.0 * (double)N * N * N), S);
    return hipGetLastError();
}

hipError_t launch_fill_random(bool f64, void* p, long long nreal, unsigned long long seed, hipStream_t s)
{
    if (nreal <= 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_fill_random<double>, dim3(nblocks(nreal, 256)), dim3(256), 0, s, (double*)p, nreal, seed);
    else hipLaunchKernelGGL(k_fill_random<float>, dim3(nblocks(nreal, 256)), dim3(256), 0, s, (float*)p, nreal, seed);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace ns
