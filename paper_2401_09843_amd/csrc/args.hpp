// Kernel argument blocks and the per-size launcher table shared by the pass
// kernels (passes.hpp, instantiated per grid size) and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ns {

// Compact retained-mode arrays (spectral states, the adjoint's strain): per
// sample, nc components of the M retained k_z rows of the MMx = M Mx columns
// s = j_y Mx + k_x.  Columns are stored in blocks of CB neighbours, CB = 64
// bytes of elements (8 FP32 or 4 FP64 complex values): element (component
// c, row jz, column s) of a sample lies at
//     (s / CB) nc M CB + c M CB + jz CB + s % CB,
// and a sample holds nc M MMxp elements, MMxp = MMx rounded up to CB (the
// columns beyond MMx are padding, never read as data).  A z pass over a
// tile of neighbouring columns then reads and writes whole blocks, which
// are contiguous from one row to the next.
__host__ __device__ constexpr int compact_cb(int elem_bytes) { return 64 / elem_bytes; }
__host__ __device__ constexpr int compact_cbl(int elem_bytes) { return elem_bytes == 8 ? 3 : 2; }  // log2 CB
__host__ __device__ constexpr long long compact_cols(long long MMx, int elem_bytes)
{
    return (MMx + compact_cb(elem_bytes) - 1) / compact_cb(elem_bytes) * compact_cb(elem_bytes);
}
// offset of (component c, row jz, column s) within one sample
__host__ __device__ constexpr long long compact_off(int elem_bytes, int nc, int M, int c, int jz, long long s)
{
    return (s >> compact_cbl(elem_bytes)) * ((long long)nc * M * compact_cb(elem_bytes)) +
           (long long)c * M * compact_cb(elem_bytes) + (long long)jz * compact_cb(elem_bytes) +
           (s & (compact_cb(elem_bytes) - 1));
}

// Strided-axis C2C pass over columns.  Column q of Q: outer = q / S,
// inner = q % S, and outer splits into sample b = outer / nc and plane
// c = outer % nc; element (row r) of the column lives at
// base + b * ss + c * cs + r * S + inner (complex elements).  An input in
// the compact layout (in_cbl > 0) is addressed instead as
// base + b * in_ss + c * in_cs + (inner >> in_cbl) * in_bs + r * in_rs
// + (inner & (2^in_cbl - 1)).
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
    long long in_bs = 0, in_rs = 0;  // input column-block / row strides (in_cbl > 0)
    int in_cbl = 0;                  // log2 of the input column block, 0: plain rows of S
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
// Columns are the (k_y, k_x) pairs s of the compact layout, MMx = M * Mx
// per sample, enumerated as batch * MMxp (MMxp = compact_cols(MMx)); the
// padding columns s >= MMx are skipped.  States are compact arrays of 3
// components.
struct F3Args {
    const void* in;            // [batch][ncomp][N][MMx]
    const void* u0;            // compact state u^n (may be null)
    const void* us;            // compact stage state
    void* out;                 // compact
    const void* tw;
    const void* rate;          // eps |k|^{2s} Q(|k|), indexed by |k|^2
    const double* dt;          // [batch] on the device
    long long Q;               // batch * MMxp
    int MMx, Mx, K, M;
    long long in_ss, in_cs;    // input sample / component strides
    long long st_ss, st_cs;    // state sample stride (3 M MMxp) and component stride in a block (M CB)
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

// z-inverse pass of the adjoint's vector-Jacobian product: from the compact
// adjoint state lam and velocity u (3 components each, column-blocked), the
// five stored components of the trace-free strain of P lam and the three of
// u, zero-padded to N rows and transformed along z, written as plain rows
// [batch][8][N][MMx] (sample / component strides out_ss / out_cs).  Columns
// are enumerated as batch * MMxp like the z pass.
struct StrainZArgs {
    const void* lam;
    const void* u;
    void* out;
    const void* tw;
    long long Q;               // batch * MMxp
    int MMx, Mx, K, M;
    long long st_ss, st_cs;    // compact sample stride (3 M MMxp) and component stride in a block (M CB)
    long long out_ss, out_cs;  // 8 N MMx, N MMx
};

// Schedule variants of the tuned passes.
constexpr int NS_MAXV = 16;
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
    hipError_t (*strain_z)(const StrainZArgs&, hipStream_t);  // strain of P lam (5) and u (3), inverse z
    hipError_t (*x_adj)(const XArgs&, hipStream_t);     // C2R of S (5) and u (3), a = 2 S u, R2C
    hipError_t (*f3_adj)(const F3Args&, hipStream_t);   // z forward of 3 comps + adjoint epilogue
    const char* desc;
};

const SizeKernels* find_kernels(int N, bool f64);
int supported_sizes(int* out, int cap);

}  // namespace ns
