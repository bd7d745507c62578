// Kernels for grid size N = 256 (FP32 and FP64), with the schedule variants
// the autotuner chooses from.
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<256, 16, Radices<16, 16>>;
using PB = Plan<256, 32, Radices<8, 8, 4>>;
using PBR = Plan<256, 32, Radices<4, 8, 8>>;
using PC = Plan<256, 64, Radices<4, 4, 4, 4>>;
using PH = Plan<128, 16, Radices<8, 2, 8>>;  // half-length x lines

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<256, R>::make();  // col: PA T16; x: PB U2; f3: PB T8
    add_col<PA, 32, 0, 1, R>(k, "G16 r16.16 T32");
    add_col<PA, 64, 0, 1, R>(k, "G16 r16.16 T64");
    add_col<PB, 16, 0, 1, R>(k, "G32 r8.8.4 T16");
    add_col<PB, 32, 0, 1, R>(k, "G32 r8.8.4 T32");
    add_col_p<PA, 16, 0, 1, 4, R>(k, "persistent G16 r16.16 T16 x4");
    add_col_p<PA, 32, 0, 1, 2, R>(k, "persistent G16 r16.16 T32 x2");
    add_x<PB, PBR, 4, 1, R>(k, "G32 r8.8.4 U4");
    add_x<PB, PBR, 8, 1, R>(k, "G32 r8.8.4 U8");
    add_x<PA, PA, 4, 1, R>(k, "G16 r16.16 U4");
    add_x<PA, PA, 8, 1, R>(k, "G16 r16.16 U8");
    add_x_ws<PB, PBR, 4, 1, R>(k, "G32 r8.8.4 U4 wave");
    add_x_ws<PA, PA, 8, 1, R>(k, "G16 r16.16 U8 wave");
    add_xh<PH, 16, 1, R>(k, "half G16 r8.2.8 U16");
    add_f3<PB, 4, 0, 1, R>(k, "G32 r8.8.4 T4");
    add_f3<PB, 16, 0, 1, R>(k, "G32 r8.8.4 T16");
    add_f3<PA, 16, 0, 1, R>(k, "G16 r16.16 T16");
    add_f3<PC, 4, 0, 1, R>(k, "G64 r4.4.4.4 T4");
    add_f3<PB, 16, 0, 1, R, 1>(k, "G32 r8.8.4 T16 prefetch");
    add_f3<PB, 32, 0, 1, R, 1>(k, "G32 r8.8.4 T32 prefetch");
    return k;
}

SizeKernels make64()
{
    using R = double;
    SizeKernels k = Launch<256, R>::make();
    add_col<PA, 16, 0, 1, R>(k, "G16 r16.16 T16");
    add_x<PB, PBR, 4, 1, R>(k, "G32 r8.8.4 U4");
    add_f3<PB, 8, 0, 1, R>(k, "G32 r8.8.4 T8");
    return k;
}
}  // namespace

const SizeKernels* kernels_256(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = make64();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
