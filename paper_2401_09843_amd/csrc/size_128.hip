// Kernels for grid size N = 128 (FP32 and FP64), with the schedule variants
// the autotuner chooses from.
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<128, 8, Radices<16, 8>>;
using PB = Plan<128, 16, Radices<8, 8, 2>>;
using PBR = Plan<128, 16, Radices<2, 8, 8>>;
using PC = Plan<128, 32, Radices<4, 4, 4, 2>>;
using PCR = Plan<128, 32, Radices<2, 4, 4, 4>>;
using PH = Plan<64, 8, Radices<8, 8>>;  // half-length x lines
using PS = Plan<128, 16, Radices<8, 2, 8>>;  // one plan for both x-pass halves

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<128, R>::make();  // col: PA T16; x: PB U4; f3: PB T16
    add_col<PA, 32, 0, 1, R>(k, "G8 r16.8 T32");
    add_col<PA, 64, 0, 1, R>(k, "G8 r16.8 T64");
    add_col<PC, 16, 0, 1, R>(k, "G32 r4.4.4.2 T16");
    add_col<PS, 32, 0, 1, R>(k, "G16 r8.2.8 T32");
    add_col<PS, 64, 0, 1, R>(k, "G16 r8.2.8 T64");
    add_col<PA, 64, 1, 1, R>(k, "G8 r16.8 T64 split");
    add_col<PA, 128, 1, 1, R>(k, "G8 r16.8 T128 split");
    add_x<PB, PBR, 8, 1, R>(k, "G16 r8.8.2 U8");
    add_x_sht<PB, PBR, 8, 1, R>(k, "G16 r8.8.2 U8 sht");
    add_x_sht<PB, PBR, 8, 1, R, false, 2>(k, "G16 r8.8.2 U8 sht2");
    add_x_sht<PS, PS, 8, 1, R>(k, "G16 r8.2.8 U8 sht");
    add_x_sht<PS, PS, 8, 1, R, false, 2>(k, "G16 r8.2.8 U8 sht2");
    add_x_sht<PS, PS, 8, 1, R, true, 3>(k, "G16 r8.2.8 U8 wave sht2 mirror");
    add_x_sht<PS, PS, 8, 1, R, false, 3>(k, "G16 r8.2.8 U8 sht2 mirror");
    add_x_sht<PS, PS, 8, 1, R, true, 2>(k, "G16 r8.2.8 U8 wave sht2");
    add_x<PC, PCR, 4, 1, R>(k, "G32 r4.4.4.2 U4");
    add_x<PA, Plan<128, 8, Radices<8, 16>>, 16, 1, R>(k, "G8 r16.8 U16");
    add_x_ws<PB, PBR, 8, 1, R>(k, "G16 r8.8.2 U8 wave");
    add_x_ws<PA, Plan<128, 8, Radices<8, 16>>, 16, 1, R>(k, "G8 r16.8 U16 wave");
    add_x_ws<PC, PCR, 4, 1, R>(k, "G32 r4.4.4.2 U4 wave");
    add_xh<PH, 16, 1, R>(k, "half G8 r8.8 U16");
    add_xh<PH, 32, 1, R>(k, "half G8 r8.8 U32");
    add_f3<PB, 8, 0, 1, R>(k, "G16 r8.8.2 T8");
    add_f3<PA, 16, 0, 1, R>(k, "G8 r16.8 T16");
    add_f3<PC, 8, 0, 1, R>(k, "G32 r4.4.4.2 T8");
    add_f3<PB, 16, 0, 1, R, 1>(k, "G16 r8.8.2 T16 prefetch");
    add_f3<PS, 16, 0, 1, R, 1>(k, "G16 r8.2.8 T16 prefetch");
    add_f3<PS, 16, 0, 1, R, 1, 1>(k, "G16 r8.2.8 T16 prefetch db");
    add_f3<PS, 8, 0, 1, R, 1>(k, "G16 r8.2.8 T8 prefetch");
    add_f3<PS, 32, 0, 1, R, 1>(k, "G16 r8.2.8 T32 prefetch");
    add_f3<PS, 64, 0, 1, R, 1>(k, "G16 r8.2.8 T64 prefetch");
    // the adjoint x pass holds eight fields per thread: four elements each;
    // its three forward transforms grouped, with the register unpack
    k.x_adj = launch_x<PC, PCR, 4, X_ADJ, 1, R, 0, false, 3>;
    return k;
}

SizeKernels make64()
{
    using R = double;
    SizeKernels k = Launch<128, R>::make();
    add_col<PA, 8, 0, 1, R>(k, "G8 r16.8 T8");
    add_col<PC, 8, 0, 1, R>(k, "G32 r4.4.4.2 T8");
    add_x<PC, PCR, 4, 1, R>(k, "G32 r4.4.4.2 U4");
    add_f3<PB, 4, 0, 1, R>(k, "G16 r8.8.2 T4");
    add_f3<PC, 4, 0, 1, R>(k, "G32 r4.4.4.2 T4");
    // the adjoint x pass holds eight fields per thread: four elements each;
    // its three forward transforms grouped, with the register unpack
    k.x_adj = launch_x<PC, PCR, 4, X_ADJ, 1, R, 0, false, 3>;
    return k;
}
}  // namespace

const SizeKernels* kernels_128(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = make64();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
