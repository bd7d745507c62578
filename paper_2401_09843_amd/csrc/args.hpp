// Kernel argument blocks and the per-size launcher table shared by the pass
// kernels (passes.hpp, instantiated per grid size) and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ns {

// Strided-axis C2C pass over columns.  Column q of Q: outer = q / S,
// inner = q % S; element (row r) of the column lives at
// base + outer * outer_stride + r * S + inner (complex elements).
struct ColArgs {
    const void* in;
    void* out;
    const void* tw;          // exp(-2 pi i e / N), N entries
    long long Q;             // number of columns
    long long S;             // contiguous columns per outer block
    long long in_os, out_os; // outer strides (complex elements)
    int K, M;                // 2/3 cutoff and compact length 2K+1
    double scale;            // output scale (forward passes)
};

// x-line pass over pairs of lines.  Line l of a sample is row l of
// [comp][N*N][row_len] arrays; unit u handles lines 2u and 2u+1.
struct XArgs {
    const void* in;
    void* out;
    const void* tw;
    long long nunits;          // batch * N * N / 2
    long long in_cs, out_cs;   // component strides (scalar or complex elements)
    long long in_ss, out_ss;   // sample strides
    int K;
    double scale;
};

// z-axis forward pass fused with the right-hand-side / projection epilogue.
// Columns are the (k_y, k_x) pairs of the compact layout, MMx = M * Mx per
// sample.
struct F3Args {
    const void* in;            // [batch][ncomp][N][MMx]
    const void* u0;            // compact state u^n   [batch][3][M][MMx] (may be null)
    const void* us;            // compact stage state [batch][3][M][MMx]
    void* out;                 // compact             [batch][3][M][MMx]
    const void* tw;
    const void* rate;          // eps |k|^{2s} Q(|k|), indexed by |k|^2
    const double* dt;          // [batch] on the device
    long long Q;               // batch * MMx
    int MMx, Mx, K, M;
    long long in_ss, in_cs;    // input sample / component strides
    long long st_ss, st_cs;    // state sample / component strides
    double ca, cb, cc;         // out = ca u0 + cb us + cc dt F
    double scale;
};

// Launchers for one grid size and precision.
struct SizeKernels {
    int N;
    hipError_t (*col_inv)(const ColArgs&, hipStream_t);   // zero-pad compact rows M -> N, inverse
    hipError_t (*col_fwd)(const ColArgs&, hipStream_t);   // forward, keep the M retained rows
    hipError_t (*x_rhs)(const XArgs&, hipStream_t);       // C2R of u, six products, R2C
    hipError_t (*x_fwd3)(const XArgs&, hipStream_t);      // R2C of a real 3-component field
    hipError_t (*x_inv3)(const XArgs&, hipStream_t);      // C2R to a real 3-component field
    hipError_t (*f3_rhs)(const F3Args&, hipStream_t);     // z forward of 6 comps + RHS / RK epilogue
    hipError_t (*f3_proj)(const F3Args&, hipStream_t);    // z forward of 3 comps + projection
    const char* desc;
};

const SizeKernels* find_kernels(int N, bool f64);
int supported_sizes(int* out, int cap);

}  // namespace ns
