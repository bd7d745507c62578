// Kernels for grid size N = 8 (FP32 and FP64).
#include "sizes.hpp"

namespace ns {
const SizeKernels* kernels_8(bool f64)
{
    static const SizeKernels k32 = Launch<8, float>::make();
    static const SizeKernels k64 = Launch<8, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
