// Kernels for grid size N = 64 (FP32 and FP64), with the schedule variants
// the autotuner chooses from.
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<64, 8, Radices<8, 8>>;
using PB = Plan<64, 16, Radices<4, 4, 4>>;
using PC = Plan<64, 4, Radices<16, 4>>;
using PCR = Plan<64, 4, Radices<4, 16>>;
using PH = Plan<32, 8, Radices<4, 2, 4>>;  // half-length x lines

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<64, R>::make();  // col: PA T16; x: PA U8; f3: PA T16
    add_col<PA, 32, 0, 1, R>(k, "G8 r8.8 T32");
    add_col<PA, 64, 0, 1, R>(k, "G8 r8.8 T64");
    add_col<PB, 16, 0, 1, R>(k, "G16 r4.4.4 T16");
    add_x<PA, PA, 16, 1, R>(k, "G8 r8.8 U16");
    add_x<PB, PB, 8, 1, R>(k, "G16 r4.4.4 U8");
    add_x<PC, PCR, 32, 1, R>(k, "G4 r16.4 U32");
    add_x_ws<PA, PA, 16, 1, R>(k, "G8 r8.8 U16 wave");
    add_x_ws<PB, PB, 8, 1, R>(k, "G16 r4.4.4 U8 wave");
    add_xh<PH, 16, 1, R>(k, "half G8 r4.2.4 U16");
    add_xh<PH, 32, 1, R>(k, "half G8 r4.2.4 U32");
    add_f3<PA, 8, 0, 1, R>(k, "G8 r8.8 T8");
    add_f3<PA, 32, 0, 1, R>(k, "G8 r8.8 T32");
    add_f3<PB, 8, 0, 1, R>(k, "G16 r4.4.4 T8");
    add_f3<PA, 32, 0, 1, R, 1>(k, "G8 r8.8 T32 prefetch");
    add_f3<PA, 64, 0, 1, R, 1>(k, "G8 r8.8 T64 prefetch");
    add_f3<PA, 128, 0, 1, R, 1>(k, "G8 r8.8 T128 prefetch");
    return k;
}

SizeKernels make64()
{
    using R = double;
    SizeKernels k = Launch<64, R>::make();
    add_col<PA, 8, 0, 1, R>(k, "G8 r8.8 T8");
    add_f3<PA, 4, 0, 1, R>(k, "G8 r8.8 T4");
    return k;
}
}  // namespace

const SizeKernels* kernels_64(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = make64();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
