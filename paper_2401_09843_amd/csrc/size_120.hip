// Kernels for grid size N = 120 (FP32 and FP64).
#include "sizes.hpp"

namespace ns {
const SizeKernels* kernels_120(bool f64)
{
    static const SizeKernels k32 = Launch<120, float>::make();
    static const SizeKernels k64 = Launch<120, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
