// Kernels for grid size N = 384 (FP32 and FP64): the padded grid 3n/2 of
// an n = 256 mode state, with the schedule variants the autotuner chooses
// from (a radix-3 or 12 stage needs E = N / G divisible by 3 and by every
// other radix: E = 24 with G = 16, E = 12 with G = 32).
#include "tuned.hpp"

namespace ns {
namespace {
using PF = Plan<384, 16, Radices<8, 4, 12>>;      // E = 24, three stages
using PX = Plan<384, 32, Radices<4, 4, 2, 12>>;   // E = 12, four stages
using PXR = Plan<384, 32, Radices<12, 2, 4, 4>>;

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<384, R>::make();  // col: r8.4.4.3; x, f3: r4.4.4.2.3
    add_col<PF, 16, 1, 1, R>(k, "G16 r8.4.12 T16 split");
    add_x<PX, PXR, 2, 1, R>(k, "G32 r4.4.2.12 U2");
    add_f3<PX, 8, 0, 1, R, 1>(k, "G32 r4.4.2.12 T8 prefetch");
    return k;
}
}  // namespace

const SizeKernels* kernels_384(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = Launch<384, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
