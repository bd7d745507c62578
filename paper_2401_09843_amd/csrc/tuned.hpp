// Helpers to register extra schedule variants of the tuned passes.
#pragma once
#include "sizes.hpp"

namespace ns {

template <class P, int T, int SP, int W, typename R>
void add_col(SizeKernels& k, const char* name)
{
    add_variant(k.inv, k.n_inv, launch_col<P, T, +1, COL_INV_PAD, SP, W, R>, name);
    add_variant(k.fwd, k.n_fwd, launch_col<P, T, -1, COL_FWD_TRUNC, SP, W, R>, name);
}

template <class P, int T, int SP, int W, int BPC, typename R>
void add_col_p(SizeKernels& k, const char* name)
{
    add_variant(k.inv, k.n_inv, launch_col_p<P, T, +1, COL_INV_PAD, SP, W, BPC, R>, name);
    add_variant(k.fwd, k.n_fwd, launch_col_p<P, T, -1, COL_FWD_TRUNC, SP, W, BPC, R>, name);
}

template <class PI, class PF, int U, int W, typename R, int BPC = 0, bool WS = false, int SHT = 0>
void add_x(SizeKernels& k, const char* name)
{
    add_variant(k.x, k.n_x, launch_x<PI, PF, U, X_RHS, W, R, BPC, WS, SHT>, name);
}

// the product x pass with transforms grouped to share twiddle reads: the
// three inverse ones (SHT = 1), and the forward ones too (SHT = 2)
template <class PI, class PF, int U, int W, typename R, bool WS = false, int SHT = 1>
void add_x_sht(SizeKernels& k, const char* name)
{
    add_variant(k.x, k.n_x, launch_x<PI, PF, U, X_RHS, W, R, 0, WS, SHT>, name);
}

// the x pass in the half-length form (one wavefront per line)
template <class PH, int U, int W, typename R, int SHT = 0>
void add_xh(SizeKernels& k, const char* name)
{
    add_variant(k.x, k.n_x, launch_xh<PH, U, W, R, SHT>, name);
}

// the x pass with wavefront-synchronous exchanges (lines of at most 64 threads)
template <class PI, class PF, int U, int W, typename R>
void add_x_ws(SizeKernels& k, const char* name)
{
    add_variant(k.x, k.n_x, launch_x<PI, PF, U, X_RHS, W, R, 0, true>, name);
}

template <class P, int T, int SP, int W, typename R, int PRE = 0, int DB = 0>
void add_f3(SizeKernels& k, const char* name)
{
    const int before = k.n_f3;
    add_variant(k.f3, k.n_f3, launch_f3<P, T, F3_RHS, SP, W, R, PRE, 0, DB>, name);
    if (k.n_f3 > before) k.f3[k.n_f3 - 1].fn_zi = launch_f3<P, T, F3_RHS, SP, W, R, PRE, 1, DB>;
}

}  // namespace ns
