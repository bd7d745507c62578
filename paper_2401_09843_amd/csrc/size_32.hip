// Kernels for grid size N = 32 (FP32 and FP64).
#include "sizes.hpp"

namespace ns {
const SizeKernels* kernels_32(bool f64)
{
    static const SizeKernels k32 = Launch<32, float>::make();
    static const SizeKernels k64 = Launch<32, double>::make();
    return f64 ? &k64 : &k32;
}
}  // namespace ns
