// Kernels for grid size N = 512 (FP32 and FP64), with the schedule variants
// the autotuner chooses from.
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<512, 64, Radices<8, 8, 8>>;
using PB = Plan<512, 32, Radices<16, 8, 4>>;
using PBR = Plan<512, 32, Radices<4, 8, 16>>;
using PC = Plan<512, 128, Radices<4, 4, 4, 4, 2>>;
using PCR = Plan<512, 128, Radices<2, 4, 4, 4, 4>>;
using PH = Plan<256, 32, Radices<8, 4, 8>>;  // half-length x lines

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<512, R>::make();  // col: PA T16; x: PA U4; f3: PA T8
    add_col<PA, 8, 0, 1, R>(k, "G64 r8.8.8 T8");
    add_col<PA, 16, 1, 1, R>(k, "G64 r8.8.8 T16 split");
    add_col<PB, 16, 0, 1, R>(k, "G32 r16.8.4 T16");
    add_col<PB, 32, 1, 1, R>(k, "G32 r16.8.4 T32 split");
    add_col_p<PA, 8, 0, 1, 2, R>(k, "persistent G64 r8.8.8 T8 x2");
    add_col_p<PA, 16, 0, 1, 1, R>(k, "persistent G64 r8.8.8 T16 x1");
    add_x<PA, PA, 2, 1, R>(k, "G64 r8.8.8 U2");
    add_x<PA, PA, 4, 3, R>(k, "G64 r8.8.8 U4 w3");
    add_x<PB, PBR, 4, 1, R>(k, "G32 r16.8.4 U4");
    add_x<PC, PCR, 2, 1, R>(k, "G128 r4.4.4.4.2 U2");
    add_x_ws<PA, PA, 2, 1, R>(k, "G64 r8.8.8 U2 wave");
    add_x_ws<PA, PA, 4, 3, R>(k, "G64 r8.8.8 U4 wave w3");
    add_x_sht<PA, PA, 4, 3, R, true>(k, "G64 r8.8.8 U4 wave w3 sht");
    add_x_sht<PA, PA, 4, 3, R, true, 2>(k, "G64 r8.8.8 U4 wave w3 sht2");
    add_x_sht<PA, PA, 2, 3, R, true, 2>(k, "G64 r8.8.8 U2 wave w3 sht2");
    add_x_sht<PA, PA, 4, 3, R, true, 3>(k, "G64 r8.8.8 U4 wave w3 sht2 mirror");
    add_x_ws<PB, PBR, 4, 1, R>(k, "G32 r16.8.4 U4 wave");
    add_xh<PH, 8, 1, R>(k, "half G32 r8.4.8 U8");
    add_f3<PA, 4, 0, 1, R>(k, "G64 r8.8.8 T4");
    add_f3<PA, 8, 1, 1, R>(k, "G64 r8.8.8 T8 split");
    add_f3<PC, 4, 0, 1, R>(k, "G128 r4.4.4.4.2 T4");
    add_f3<PB, 8, 0, 1, R>(k, "G32 r16.8.4 T8");
    add_f3<PA, 8, 0, 1, R, 1>(k, "G64 r8.8.8 T8 prefetch");
    add_f3<PA, 16, 0, 1, R, 1>(k, "G64 r8.8.8 T16 prefetch");
    add_f3<PA, 8, 0, 1, R, 1, 1>(k, "G64 r8.8.8 T8 prefetch db");
    return k;
}

SizeKernels make64()
{
    using R = double;
    SizeKernels k = Launch<512, R>::make();
    add_col<PA, 4, 0, 1, R>(k, "G64 r8.8.8 T4");
    add_x<PA, PA, 4, 1, R>(k, "G64 r8.8.8 U4");
    add_f3<PA, 2, 0, 1, R>(k, "G64 r8.8.8 T2");
    return k;
}
}  // namespace

const SizeKernels* kernels_512(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = make64();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
