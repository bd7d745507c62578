// Kernels for grid size N = 768 (FP32 and FP64): the padded grid 3n/2 of
// an n = 512 mode state, with the schedule variants the autotuner chooses
// from (a radix-3, 6 or 12 stage needs E = N / G divisible by 3 and by every
// other radix: E = 24 with G = 32, E = 12 with G = 64).
#include "tuned.hpp"

namespace ns {
namespace {
using PA = Plan<768, 32, Radices<8, 8, 4, 3>>;
using PB = Plan<768, 64, Radices<4, 4, 4, 4, 3>>;
using PF = Plan<768, 32, Radices<8, 8, 12>>;      // E = 24, three stages
using PX = Plan<768, 64, Radices<4, 4, 4, 12>>;   // E = 12, four stages
using PXR = Plan<768, 64, Radices<12, 4, 4, 4>>;

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<768, R>::make();  // col: PA T16; x: PB U2; f3: PB T8
    add_col<PA, 16, 1, 1, R>(k, "G32 r8.8.4.3 T16 split");
    add_col<PA, 8, 1, 1, R>(k, "G32 r8.8.4.3 T8 split");
    add_col<PB, 16, 1, 1, R>(k, "G64 r4.4.4.4.3 T16 split");
    add_col<PF, 16, 1, 1, R>(k, "G32 r8.8.12 T16 split");
    add_x<PX, PXR, 2, 1, R>(k, "G64 r4.4.4.12 U2");
    add_f3<PB, 8, 0, 1, R, 1>(k, "G64 r4.4.4.4.3 T8 prefetch");
    add_f3<PX, 8, 0, 1, R, 1>(k, "G64 r4.4.4.12 T8 prefetch");
    add_f3<PB, 8, 1, 1, R, 1>(k, "G64 r4.4.4.4.3 T8 split prefetch");
    return k;
}
}  // namespace

const SizeKernels* kernels_768(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = Launch<768, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
