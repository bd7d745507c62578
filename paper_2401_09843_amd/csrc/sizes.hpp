// Built-in FFT schedules per grid size N.  Column passes: G threads per
// line, radices Rad; x pass: GX threads per line, radices XRad for the
// inverse and XRadRev for the forward half; fused z pass: GF threads,
// radices FRad.  T / TF: columns per block of the column / fused z passes,
// U: line pairs per block of the x pass (FP32, FP64).
#pragma once
#include "passes.hpp"

namespace ns {

#define NS_R(...) __VA_ARGS__
#define NS_SIZE_CFG(NN, GG, RAD, GXX, XRAD, XRADREV, GFF, FRAD, T32_, T64_, TF32_, TF64_, U32_, U64_, SP32_, SP64_, \
                    SPF32_, SPF64_)                                                                 \
    template <>                                                                                    \
    struct SizeCfg<NN> {                                                                           \
        static constexpr int G = GG, GX = GXX, GF = GFF;                                           \
        using Rad = Radices<RAD>;                                                                  \
        using XRad = Radices<XRAD>;                                                                \
        using XRadRev = Radices<XRADREV>;                                                          \
        using FRad = Radices<FRAD>;                                                                \
        static constexpr int T32 = T32_, T64 = T64_, TF32 = TF32_, TF64 = TF64_;                   \
        static constexpr int U32 = U32_, U64 = U64_;                                               \
        static constexpr int SP32 = SP32_, SP64 = SP64_, SPF32 = SPF32_, SPF64 = SPF64_;           \
        static constexpr const char* desc = "N=" #NN;                                              \
    };

//            N   G  Rad                  GX XRad                  XRadRev               GF FRad                 T32 T64 TF32 TF64 U32 U64 SP32 SP64 SPF32 SPF64
NS_SIZE_CFG(8,    1, NS_R(8),             1, NS_R(8),              NS_R(8),              1, NS_R(8),             64, 32, 32, 16, 64, 32, 0, 0, 0, 0)
NS_SIZE_CFG(12,   1, NS_R(4, 3),          1, NS_R(4, 3),           NS_R(3, 4),           1, NS_R(4, 3),          64, 32, 32, 16, 64, 32, 0, 0, 0, 0)
NS_SIZE_CFG(16,   4, NS_R(4, 4),          4, NS_R(4, 4),           NS_R(4, 4),           4, NS_R(4, 4),          32, 16, 32, 16, 16, 16, 0, 0, 0, 0)
NS_SIZE_CFG(20,   1, NS_R(4, 5),          1, NS_R(4, 5),           NS_R(5, 4),           1, NS_R(4, 5),          64, 32, 32, 16, 64, 32, 0, 0, 0, 0)
NS_SIZE_CFG(24,   2, NS_R(4, 2, 3),       2, NS_R(4, 2, 3),        NS_R(3, 2, 4),        2, NS_R(4, 2, 3),       32, 16, 32, 16, 32, 16, 0, 0, 0, 0)
NS_SIZE_CFG(32,   4, NS_R(8, 4),          4, NS_R(8, 4),           NS_R(4, 8),           4, NS_R(8, 4),          32, 16, 16, 16, 16, 16, 0, 0, 0, 0)
NS_SIZE_CFG(40,   2, NS_R(2, 4, 5),       2, NS_R(2, 4, 5),        NS_R(5, 4, 2),        2, NS_R(2, 4, 5),       32, 16, 16, 8, 32, 16, 0, 0, 0, 0)
NS_SIZE_CFG(48,   4, NS_R(4, 4, 3),       4, NS_R(4, 4, 3),        NS_R(3, 4, 4),        4, NS_R(4, 4, 3),       32, 16, 16, 8, 16, 16, 0, 0, 0, 0)
NS_SIZE_CFG(60,   2, NS_R(2, 2, 3, 5),    2, NS_R(2, 2, 3, 5),     NS_R(5, 3, 2, 2),     2, NS_R(2, 2, 3, 5),    32, 16, 16, 8, 32, 16, 0, 0, 0, 0)
NS_SIZE_CFG(64,   8, NS_R(8, 8),          8, NS_R(8, 8),           NS_R(8, 8),           8, NS_R(8, 8),          16, 16, 16, 8, 8, 8, 0, 0, 0, 0)
NS_SIZE_CFG(80,   4, NS_R(4, 4, 5),       4, NS_R(4, 4, 5),        NS_R(5, 4, 4),        4, NS_R(4, 4, 5),       16, 16, 16, 8, 16, 8, 0, 0, 0, 0)
NS_SIZE_CFG(96,   8, NS_R(4, 2, 4, 3),    8, NS_R(4, 2, 4, 3),     NS_R(3, 4, 2, 4),     8, NS_R(4, 2, 4, 3),    16, 16, 16, 8, 8, 8, 0, 0, 0, 0)
NS_SIZE_CFG(120,  4, NS_R(2, 2, 2, 3, 5), 4, NS_R(2, 2, 2, 3, 5),  NS_R(5, 3, 2, 2, 2),  4, NS_R(2, 2, 2, 3, 5), 16, 8, 16, 8, 16, 8, 0, 0, 0, 0)
NS_SIZE_CFG(128,  8, NS_R(16, 8),         16, NS_R(8, 8, 2),       NS_R(2, 8, 8),        16, NS_R(8, 8, 2),      16, 16, 16, 8, 4, 4, 0, 0, 0, 0)
NS_SIZE_CFG(256,  16, NS_R(16, 16),       32, NS_R(8, 8, 4),       NS_R(4, 8, 8),        32, NS_R(8, 8, 4),      16, 8, 8, 4, 2, 2, 0, 0, 0, 0)
NS_SIZE_CFG(512,  64, NS_R(8, 8, 8),      64, NS_R(8, 8, 8),       NS_R(8, 8, 8),        64, NS_R(8, 8, 8),      16, 8, 8, 4, 4, 2, 0, 0, 0, 0)
NS_SIZE_CFG(1024, 64, NS_R(16, 16, 4),    128, NS_R(8, 8, 4, 4),   NS_R(4, 4, 8, 8),     128, NS_R(8, 8, 4, 4),  16, 8, 4, 2, 2, 1, 1, 1, 0, 0)
// the padded grids 3n/2 of n = 128, 256, 512, 1024 modes (a radix-3 stage
// needs E = N / G divisible by 3 and by every other radix)
NS_SIZE_CFG(192,  16, NS_R(4, 4, 4, 3),   16, NS_R(4, 4, 4, 3),    NS_R(3, 4, 4, 4),     16, NS_R(4, 4, 4, 3),   16, 8, 8, 4, 4, 2, 0, 0, 0, 0)
NS_SIZE_CFG(384,  16, NS_R(8, 4, 4, 3),   32, NS_R(4, 4, 4, 2, 3), NS_R(3, 2, 4, 4, 4),  32, NS_R(4, 4, 4, 2, 3), 16, 8, 8, 4, 2, 2, 0, 0, 0, 0)
NS_SIZE_CFG(768,  32, NS_R(8, 8, 4, 3),   64, NS_R(4, 4, 4, 4, 3), NS_R(3, 4, 4, 4, 4),  64, NS_R(4, 4, 4, 4, 3), 16, 8, 8, 4, 2, 1, 0, 0, 0, 0)
NS_SIZE_CFG(1536, 64, NS_R(8, 8, 8, 3),   128, NS_R(4, 4, 4, 4, 2, 3), NS_R(3, 2, 4, 4, 4, 4), 128, NS_R(4, 4, 4, 4, 2, 3), 8, 4, 4, 2, 1, 1, 0, 0, 0, 0)
#undef NS_SIZE_CFG
#undef NS_R

}  // namespace ns
