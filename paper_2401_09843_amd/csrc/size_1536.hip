// Kernels for grid size N = 1536 (FP32 and FP64): the padded grid 3n/2 of
// an n = 1024 mode state, with the schedule variants the autotuner chooses
// from.  A radix-3 or 12 stage needs E = N / G divisible by 3 and by every
// other radix, so lines use E = 12 (G = 128) or E = 24 (G = 64).
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<1536, 64, Radices<8, 8, 8, 3>>;
using PB = Plan<1536, 128, Radices<4, 4, 4, 4, 2, 3>>;
using PBR = Plan<1536, 128, Radices<3, 2, 4, 4, 4, 4>>;
using PX = Plan<1536, 128, Radices<4, 4, 4, 2, 12>>;   // E = 12, five stages
using PXR = Plan<1536, 128, Radices<12, 2, 4, 4, 4>>;

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<1536, R>::make();  // col: PA T8; x: PB U1; f3: PB T4
    add_col<PA, 8, 1, 1, R>(k, "G64 r8.8.8.3 T8 split");
    add_col<PB, 8, 0, 1, R>(k, "G128 r4.4.4.4.2.3 T8");
    add_x<PB, PBR, 2, 1, R>(k, "G128 r4.4.4.4.2.3 U2");
    add_x<PX, PXR, 2, 1, R>(k, "G128 r4.4.4.2.12 U2");
    add_f3<PX, 4, 0, 1, R, 1>(k, "G128 r4.4.4.2.12 T4 prefetch");
    add_f3<PB, 4, 0, 1, R, 1>(k, "G128 r4.4.4.4.2.3 T4 prefetch");
    add_f3<PB, 4, 1, 1, R, 1>(k, "G128 r4.4.4.4.2.3 T4 split prefetch");
    return k;
}
}  // namespace

const SizeKernels* kernels_1536(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = Launch<1536, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
