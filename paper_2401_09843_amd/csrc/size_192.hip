// Kernels for grid size N = 192 (FP32 and FP64): the padded grid 3n/2 of
// an n = 128 mode state, with the schedule variants the autotuner chooses
// from (E = 12 with G = 16 fits radix 12: three stages).
#include "tuned.hpp"

namespace ns {
namespace {
using PX = Plan<192, 16, Radices<4, 4, 12>>;
using PXR = Plan<192, 16, Radices<12, 4, 4>>;

SizeKernels make32()
{
    using R = float;
    SizeKernels k = Launch<192, R>::make();  // col, x, f3: r4.4.4.3
    add_col<PX, 16, 1, 1, R>(k, "G16 r4.4.12 T16 split");
    add_x<PX, PXR, 4, 1, R>(k, "G16 r4.4.12 U4");
    add_f3<PX, 8, 0, 1, R, 1>(k, "G16 r4.4.12 T8 prefetch");
    return k;
}
}  // namespace

const SizeKernels* kernels_192(bool f64)
{
    static const SizeKernels k32 = make32();
    static const SizeKernels k64 = Launch<192, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
