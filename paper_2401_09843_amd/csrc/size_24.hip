// Kernels for grid size N = 24 (FP32 and FP64).
#include "sizes.hpp"

namespace ns {
const SizeKernels* kernels_24(bool f64)
{
    static const SizeKernels k32 = Launch<24, float>::make();
    static const SizeKernels k64 = Launch<24, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
