// Kernels for grid size N = 1024 (FP32 and FP64), with the schedule
// variants the autotuner chooses from.
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<1024, 64, Radices<16, 16, 4>>;
using PB = Plan<1024, 128, Radices<8, 8, 4, 4>>;
using PBR = Plan<1024, 128, Radices<4, 4, 8, 8>>;
using PC = Plan<1024, 64, Radices<16, 16, 4>>;
using PCR = Plan<1024, 64, Radices<4, 16, 16>>;
using PD = Plan<1024, 256, Radices<4, 4, 4, 4, 4>>;
using PE = Plan<1024, 128, Radices<4, 8, 8, 4>>;
using PAR = Plan<1024, 64, Radices<4, 16, 16>>;
using PH = Plan<512, 64, Radices<8, 8, 8>>;  // half-length x lines
using PS = Plan<1024, 128, Radices<8, 4, 4, 8>>;  // one plan (and twiddle table) for both x-pass halves

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<1024, R>::make();  // col: PA T16 split; x: PB U2; f3: PB T4
    add_col<PA, 8, 0, 1, R>(k, "G64 r16.16.4 T8");
    add_col<PA, 16, 0, 1, R>(k, "G64 r16.16.4 T16");
    add_col<PB, 8, 0, 1, R>(k, "G128 r8.8.4.4 T8");
    add_col<PB, 8, 1, 1, R>(k, "G128 r8.8.4.4 T8 split");
    add_col<PS, 8, 0, 1, R>(k, "G128 r8.4.4.8 T8");
    add_col<PS, 8, 1, 1, R>(k, "G128 r8.4.4.8 T8 split");
    add_col_p<PA, 8, 0, 1, 2, R>(k, "persistent G64 r16.16.4 T8 x2");
    add_col_p<PA, 8, 1, 1, 2, R>(k, "persistent G64 r16.16.4 T8 split x2");
    add_col_p<PB, 8, 1, 1, 2, R>(k, "persistent G128 r8.8.4.4 T8 split x2");
    add_x<PB, PBR, 2, 3, R>(k, "G128 r8.8.4.4 U2 w3");
    add_x<PB, PBR, 2, 4, R>(k, "G128 r8.8.4.4 U2 w4");
    add_x<PE, PE, 2, 4, R>(k, "G128 r4.8.8.4 U2 w4");
    add_x_sht<PB, PBR, 2, 4, R>(k, "G128 r8.8.4.4 U2 w4 sht");
    add_x_sht<PB, PBR, 2, 4, R, false, 2>(k, "G128 r8.8.4.4 U2 w4 sht2");
    add_x_sht<PE, PE, 2, 4, R, false, 2>(k, "G128 r4.8.8.4 U2 w4 sht2");
    add_x_sht<PE, PE, 2, 4, R>(k, "G128 r4.8.8.4 U2 w4 sht");
    add_x_sht<PS, PS, 1, 4, R, false, 2>(k, "G128 r8.4.4.8 U1 w4 sht2");
    add_x_sht<PS, PS, 2, 4, R, false, 2>(k, "G128 r8.4.4.8 U2 w4 sht2");
    add_x_sht<PS, PS, 1, 4, R, false, 3>(k, "G128 r8.4.4.8 U1 w4 sht2 mirror");
    add_x_sht<PS, PS, 2, 4, R, false, 3>(k, "G128 r8.4.4.8 U2 w4 sht2 mirror");
    add_x<PB, PBR, 2, 4, R, 4>(k, "persistent G128 r8.8.4.4 U2 w4 x4");
    add_xh<PH, 4, 1, R>(k, "half G64 r8.8.8 U4");
    add_xh<PH, 4, 4, R>(k, "half G64 r8.8.8 U4 w4");
    add_xh<PH, 4, 4, R, 2>(k, "half G64 r8.8.8 U4 w4 sht2");
    add_f3<PB, 4, 1, 1, R, 1>(k, "G128 r8.8.4.4 T4 split prefetch");
    add_f3<PB, 8, 0, 1, R, 1>(k, "G128 r8.8.4.4 T8 prefetch");
    add_f3<PE, 8, 0, 1, R, 1>(k, "G128 r4.8.8.4 T8 prefetch");
    add_f3<PB, 8, 1, 1, R, 1>(k, "G128 r8.8.4.4 T8 split prefetch");
    add_f3<PC, 8, 1, 1, R>(k, "G64 r16.16.4 T8 split");
    add_f3<PD, 4, 0, 1, R, 1>(k, "G256 r4.4.4.4.4 T4 prefetch");
    // double-buffered exchanges: one barrier per exchange
    add_f3<PB, 8, 0, 1, R, 1, 1>(k, "G128 r8.8.4.4 T8 prefetch db");
    add_f3<PS, 8, 0, 1, R, 1, 1>(k, "G128 r8.4.4.8 T8 prefetch db");
    return k;
}

SizeKernels make64()
{
    using R = double;
    SizeKernels k = Launch<1024, R>::make();
    add_col<PA, 8, 1, 1, R>(k, "G64 r16.16.4 T8 split");
    add_col<PB, 4, 0, 1, R>(k, "G128 r8.8.4.4 T4");
    add_x<PB, PBR, 2, 1, R>(k, "G128 r8.8.4.4 U2");
    add_f3<PB, 2, 1, 1, R>(k, "G128 r8.8.4.4 T2 split");
    return k;
}
}  // namespace

const SizeKernels* kernels_1024(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = make64();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
