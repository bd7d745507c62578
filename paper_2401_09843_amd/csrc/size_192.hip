// Kernels for grid size N = 192 (FP32 and FP64): the padded grid 3n/2 of
// an n = 128 mode state.
#include "sizes.hpp"

namespace ns {
const SizeKernels* kernels_192(bool f64)
{
    static const SizeKernels k32 = Launch<192, float>::make();
    static const SizeKernels k64 = Launch<192, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
