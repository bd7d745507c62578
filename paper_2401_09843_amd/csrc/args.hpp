// Kernel argument blocks and the per-size launcher table shared by the pass
// kernels (passes.hpp, instantiated per grid size) and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ns {

// Strided-axis C2C pass over columns.  Column q of Q: outer = q / S,
// inner = q % S, and outer splits into sample b = outer / nc and plane
// c = outer % nc; element (row r) of the column lives at
// base + b * ss + c * cs + r * S + inner (complex elements).
struct ColArgs {
    const void* in;
    void* out;
    const void* tw;            // exp(-2 pi i e / N), N entries
    long long Q;               // number of columns
    long long S;               // contiguous columns per plane
    long long nc;              // planes per sample
    long long in_cs, in_ss;    // input plane / sample strides
    long long out_cs, out_ss;  // output plane / sample strides
    int K, M;                  // 2/3 cutoff and compact length 2K+1
    double scale;              // output scale (forward passes)
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
    // adjoint epilogue: out = ca L3 + c2 L2 + c1 L1 + cc dt (a - rate lam)
    // with L3 = u0, lam = us
    const void* l2;
    const void* l1;
    double c2, c1;
    // fused form of F3_RHS only: the inverse z transform of the new state,
    // zero-padded to N rows (the next stage's first pass), written to
    // [batch][3][N][MMx] with the input's sample / component strides; may
    // be the input itself (each column is read in full before it is written)
    void* zinv;
};

// Schedule variants of the tuned passes.
constexpr int NS_MAXV = 12;
struct ColVariant {
    hipError_t (*fn)(const ColArgs&, hipStream_t);
    const char* name;
};
struct XVariant {
    hipError_t (*fn)(const XArgs&, hipStream_t);
    const char* name;
};
struct F3Variant {
    hipError_t (*fn)(const F3Args&, hipStream_t);
    const char* name;
    hipError_t (*fn_zi)(const F3Args&, hipStream_t);  // the same schedule, also writing zinv
};

// Launchers for one grid size and precision: variant lists of the passes of
// the right-hand side (inverse column passes I1 and I2 share `inv`, F2 uses
// `fwd`), and single schedules of the transforms used at set-up.
struct SizeKernels {
    int N;
    int n_inv, n_fwd, n_x, n_f3;
    ColVariant inv[NS_MAXV];   // zero-pad compact rows M -> N, inverse
    ColVariant fwd[NS_MAXV];   // forward, keep the M retained rows
    XVariant x[NS_MAXV];       // C2R of u, six products, R2C
    F3Variant f3[NS_MAXV];     // z forward of 6 comps + RHS / RK epilogue (+ fused inverse z)
    hipError_t (*x_fwd3)(const XArgs&, hipStream_t);    // R2C of a real 3-component field
    hipError_t (*x_inv3)(const XArgs&, hipStream_t);    // C2R to a real 3-component field
    hipError_t (*f3_proj)(const F3Args&, hipStream_t);  // z forward of 3 comps + projection
    hipError_t (*x_adj)(const XArgs&, hipStream_t);     // C2R of S (6) and u (3), a = 2 S u, R2C
    hipError_t (*f3_adj)(const F3Args&, hipStream_t);   // z forward of 3 comps + adjoint epilogue
    const char* desc;
};

const SizeKernels* find_kernels(int N, bool f64);
int supported_sizes(int* out, int cap);

}  // namespace ns
