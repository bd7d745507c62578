// Kernels for grid size N = 384 (FP32 and FP64): the padded grid 3n/2 of
// an n = 256 mode state.
#include "sizes.hpp"

namespace ns {
const SizeKernels* kernels_384(bool f64)
{
    static const SizeKernels k32 = Launch<384, float>::make();
    static const SizeKernels k64 = Launch<384, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
