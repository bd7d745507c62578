// Launchers of the size-independent kernels (misc_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace ns {
hipError_t launch_pack(bool f64, const void* r2c, void* compact, int N, int K, hipStream_t s);
hipError_t launch_unpack(bool f64, const void* compact, void* r2c, int N, int K, hipStream_t s);
hipError_t launch_project(bool f64, void* r2c, int N, int K, hipStream_t s);
// kind 0: energy spectrum, 1: enstrophy spectrum
hipError_t launch_spectrum(bool f64, const void* r2c, double* E, int N, int K, int kbins, hipStream_t s, int kind = 0);
// pointwise mean and variance (1/B) of B samples [B][n], FP64, sample order
hipError_t launch_moments(bool f64, const void* x, int B, long long n, double* mean, double* var, hipStream_t s);
// pointwise 1-D Wasserstein-1 distance of two sample sets [na][npts] and
// [nb][npts] into w [npts]; mean (if non-null) [ncomp] = mean of each of the
// ncomp equal parts of w; fails if na + nb exceeds 20480
// longitudinal structure functions of B physical fields [B][3][N^3]: partial
// sums into part (B * lmax * sfun_blocks(N) doubles), then per sample b
// launch_sfun_final(part + b * lmax * sfun_blocks(N), ...) writes S[l - 1],
// l = 1..lmax
int sfun_blocks(int N);
hipError_t launch_sfun(bool f64, const void* u, int N, int lmax, int B, double p, double* part, hipStream_t s);
hipError_t launch_sfun_final(const double* part, int N, int lmax, double* S, hipStream_t s);
hipError_t launch_w1(bool f64, const void* a, int na, const void* b, int nb, long long npts, int ncomp, double* w,
                     double* mean, hipStream_t s);
hipError_t launch_fill(double* p, double v, int n, hipStream_t s);
hipError_t launch_fill_random(bool f64, void* p, long long nreal, unsigned long long seed, hipStream_t s);
}  // namespace ns
