// Pass kernels of one right-hand-side evaluation (Algorithm 2 with the
// padded inverse / unpadding forward transforms of Algorithm 3 replaced by
// pruned passes on the N^3 grid: zero rows are never stored).
//
//   I1  inverse C2C along z, compact k_z rows M -> N    (k_colfft, COL_INV_PAD)
//   I2  inverse C2C along y, compact k_y rows M -> N    (k_colfft, COL_INV_PAD)
//   X   C2R along x, six products u_i u_j, R2C along x  (k_xline, X_RHS)
//   F2  forward C2C along y, keep the M retained rows   (k_colfft, COL_FWD_TRUNC)
//   F3  forward C2C along z of the six products, then -i k.B-hat, the Leray
//       projection (eq. (2.5)), hyperviscosity (eqs. (2.1)-(2.3)) and the
//       SSP-RK3 stage combination (eq. (2.6))            (k_f3, F3_RHS);
//       its fused form (ZI = 1) also runs the next stage's I1 on the new
//       state while it is in registers
//
// Strided axes are transformed by tiles of T neighbouring columns: each
// thread loads whole rows of T columns (coalesced) straight into registers,
// and only the Stockham exchanges go through LDS.
#pragma once
#include <type_traits>

#include "args.hpp"
#include "fft_engine.hpp"

namespace ns {

enum { COL_INV_PAD = 0, COL_FWD_TRUNC = 1 };
enum { X_RHS = 0, X_FWD3 = 1, X_INV3 = 2, X_ADJ = 3 };
enum { F3_RHS = 0, F3_PROJ = 1, F3_ADJ = 2 };

// compact index of FFT row n (wavenumber n or n - N), or -1 outside |k| <= K
__device__ __forceinline__ int compact_of(int n, int N, int K, int M)
{
    return n <= K ? n : (n >= N - K ? n - N + M : -1);
}

// The 2/3-rule cutoff K = floor((N - 1) / 3) and compact length M = 2K + 1
// are fixed by N; the kernels take them as constants (the launchers reject
// arguments that disagree).
template <int N>
struct Cut {
    static constexpr int K = (N - 1) / 3, M = 2 * K + 1;
};

// Slot i of a thread's final output (row out_pos(t, i), t < G) holds a
// retained row |k_z| <= K for some thread t; slots that never do need no
// epilogue code.
template <class P>
__device__ __forceinline__ constexpr bool slot_may_keep(int i)
{
    constexpr int N = P::N, K = Cut<P::N>::K;
    const int base = (i / P::RL) * P::G + (i % P::RL) * (N / P::RL);
    return base <= K || base + P::G - 1 >= N - K;
}

// ------------------------------------------------------------------ I1/I2/F2
// LDS bytes of a column tile (complex or split exchange), 16-byte aligned
template <class P, int T, int SP, typename R>
constexpr size_t tile_bytes()
{
    return ((SP ? sizeof(R) : sizeof(cpx<R>)) * P::lds_len * T + 15) / 16 * 16;
}

// input offset of column `inner` of a plane, and the input row stride
// (plain rows of S columns, or the column blocks of the compact layout)
__device__ __forceinline__ long long col_in_off(const ColArgs& a, long long inner)
{
    return a.in_cbl ? (inner >> a.in_cbl) * a.in_bs + (inner & ((1LL << a.in_cbl) - 1)) : inner;
}
__device__ __forceinline__ long long col_in_rs(const ColArgs& a) { return a.in_cbl ? a.in_rs : a.S; }

// DB = 1 double-buffers the LDS exchanges (one barrier per exchange).
template <class P, int T, int DIR, int MODE, int SP, int W, typename R, int DB = 0>
__global__ void __launch_bounds__(P::G* T, W) k_colfft(ColArgs a)
{
    constexpr int N = P::N, E = P::E, KC = Cut<N>::K, MC = Cut<N>::M;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TB = (int)tile_bytes<P, T, SP, R>();
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* twl = reinterpret_cast<cpx<R>*>(smem_raw + (DB ? 2 : 1) * TB);
    const int tid = threadIdx.x, c = tid % T, g = tid / T;
    const long long q = xcd_tile(gridDim.x) * T + c;
    const bool valid = q < a.Q;
    const long long outer = valid ? q / a.S : 0;
    const long long inner = valid ? q % a.S : 0;
    const long long sb = outer / a.nc, pc = outer % a.nc;
    const cpx<R>* __restrict__ in = static_cast<const cpx<R>*>(a.in) + sb * a.in_ss + pc * a.in_cs + col_in_off(a, inner);
    cpx<R>* __restrict__ out = static_cast<cpx<R>*>(a.out) + sb * a.out_ss + pc * a.out_cs + inner;
    const long long irs = col_in_rs(a);

    // the column loads are issued before the twiddle tables are built, so
    // that both latencies overlap
    cpx<R> v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int n = P::in_pos(g, i);
        int r = n;
        if constexpr (MODE == COL_INV_PAD) r = compact_of(n, N, KC, MC);
        v[i] = (valid && r >= 0) ? in[r * irs] : cpx<R>{0, 0};
    }
    P::template load_tw<R>(twl, static_cast<const cpx<R>*>(a.tw));
    {
        cpx<R>* base = SP ? reinterpret_cast<cpx<R>*>(reinterpret_cast<R*>(lds) + c) : lds + c;
        int par = 0;
        if constexpr (DB) P::template run_db<DIR, T, SP>(v, g, base, twl, TB, par);
        else P::template run<DIR, T, SP>(v, g, base, twl);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int n = P::out_pos(g, i);
        if constexpr (MODE == COL_INV_PAD) {
            if (valid) out[n * a.S] = v[i];
        } else {
            const int r = compact_of(n, N, KC, MC);
            if (valid && r >= 0) out[r * a.S] = cscale(v[i], (R)a.scale);
        }
    }
}

// Persistent form: a fixed grid, each block walks a share of its XCD's
// contiguous tile range and loads the next tile into registers while it
// transforms the current one.  Every tile is handled exactly once whatever
// the hardware placement; the XCD split only decides locality.
template <class P, int T, int DIR, int MODE, int SP, int W, typename R>
__global__ void __launch_bounds__(P::G* T, W) k_colfft_p(ColArgs a)
{
    constexpr int N = P::N, E = P::E, KC = Cut<N>::K, MC = Cut<N>::M;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* twl = reinterpret_cast<cpx<R>*>(smem_raw + tile_bytes<P, T, SP, R>());
    P::template load_tw<R>(twl, static_cast<const cpx<R>*>(a.tw));
    const int tid = threadIdx.x, c = tid % T, g = tid / T;
    const long long ntiles = (a.Q + T - 1) / T;
    const long long nb = gridDim.x, x = blockIdx.x % 8, j = blockIdx.x / 8;
    const long long nbx = nb / 8 + (x < nb % 8 ? 1 : 0);
    const long long cc = ntiles / 8, rem = ntiles % 8;
    const long long start = x * cc + (x < rem ? x : rem), cnt = cc + (x < rem ? 1 : 0);

    auto column = [&](long long tile, bool& valid, long long& off_in, long long& off_out) {
        const long long q = tile * T + c;
        valid = q < a.Q;
        const long long outer = valid ? q / a.S : 0, inner = valid ? q % a.S : 0;
        const long long sb = outer / a.nc, pc = outer % a.nc;
        off_in = sb * a.in_ss + pc * a.in_cs + col_in_off(a, inner);
        off_out = sb * a.out_ss + pc * a.out_cs + inner;
    };
    auto load = [&](long long tile, cpx<R>(&v)[E]) {
        bool valid;
        long long oi, oo;
        column(tile, valid, oi, oo);
        const cpx<R>* __restrict__ in = static_cast<const cpx<R>*>(a.in) + oi;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = P::in_pos(g, i);
            int r = n;
            if constexpr (MODE == COL_INV_PAD) r = compact_of(n, N, KC, MC);
            v[i] = (valid && r >= 0) ? in[r * col_in_rs(a)] : cpx<R>{0, 0};
        }
    };
    cpx<R> v[E], vn[E];
    long long i = j;
    if (i < cnt) load(start + i, vn);
    for (; i < cnt; i += nbx) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = vn[e];
        if (i + nbx < cnt) load(start + i + nbx, vn);
        if constexpr (SP) P::template run<DIR, T, 1>(v, g, reinterpret_cast<cpx<R>*>(reinterpret_cast<R*>(lds) + c), twl);
        else P::template run<DIR, T, 0>(v, g, lds + c, twl);
        bool valid;
        long long oi, oo;
        column(start + i, valid, oi, oo);
        cpx<R>* __restrict__ out = static_cast<cpx<R>*>(a.out) + oo;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int n = P::out_pos(g, e);
            if constexpr (MODE == COL_INV_PAD) {
                if (valid) out[n * a.S] = v[e];
            } else {
                const int r = compact_of(n, N, KC, MC);
                if (valid && r >= 0) out[r * a.S] = cscale(v[e], (R)a.scale);
            }
        }
    }
}

// ------------------------------------------------------------------ X pass
// LDS elements per line of the X pass (per-stage padded exchanges)
template <class PI, class PF, typename R>
constexpr int x_line_len()
{
    constexpr int a = PI::template lds_len_st<sizeof(cpx<R>)>(), b = PF::template lds_len_st<sizeof(cpx<R>)>();
    return a > b ? a : b;
}

// The adjoint x pass parks its three transformed velocity fields in LDS
// (3 N complex values per pair of lines) when that takes at most 32 KiB per
// block, instead of holding them in registers next to the accumulators.
template <class PI, class PF, int U, typename R>
constexpr bool xadj_park()
{
    return 3 * PI::N * U * sizeof(cpx<R>) <= 32768;
}

// Two real lines l1 = 2u, l2 = 2u+1 share one complex transform: for a C2R,
// Z = A + iB with A, B the Hermitian half spectra gives z = a + i b; for an
// R2C, Z = FFT(a + i b) splits as A_k = (Z_k + conj Z_{N-k})/2,
// B_k = (Z_k - conj Z_{N-k})/(2i).
// BPC > 0 (product pass only): persistent blocks, BPC per compute unit,
// that build the twiddle tables once and then walk the tiles of U units.
// WS = true: the exchanges of a line synchronise its wavefront only (lines
// of at most 64 threads lie inside one wavefront).
// SHT (product pass) > 0: the three inverse transforms run stage by stage
// together, so each twiddle factor is read from LDS once for all three; SHT
// = 2 also groups the forward transforms of the products as xx | xy, xz |
// yy, yz, zz (each group formed once the velocity it last needs is free).
// SHT = 3 (last forward radix E): as 2, with each thread taking Z_{N-k}
// for its bins k from a lane of its own wavefront (ds_bpermute), so that
// the R2C unpack needs no LDS buffer and no barrier.  Lines of at most 64
// threads lie in one wavefront anyway; lines of 128 run the forward
// transforms' last stage in mirror_order to make it so.
template <class PI, class PF, int U, int MODE, int W, typename R, int BPC = 0, bool WS = false, int SHT = 0>
__global__ void __launch_bounds__(PI::G* U, W) k_xline(XArgs a)
{
    constexpr int N = PI::N, G = PI::G, E = PI::E;
    static_assert(PF::G == G && PF::N == N, "plans must match");
    static_assert(PF::R0 == PI::RL, "forward plan must start with the inverse plan's last radix");
    constexpr int LL = x_line_len<PI, PF, R>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* twI = reinterpret_cast<cpx<R>*>(smem_raw) + U * LL;
    // one table serves both halves when they use the same plan
    constexpr bool SAME = std::is_same<PI, PF>::value;
    cpx<R>* twF = SAME ? twI : twI + PI::tw_len;
    auto tables = [&] {
        PI::template fill_tw<R>(twI, static_cast<const cpx<R>*>(a.tw));
        if constexpr (!SAME) PF::template fill_tw<R>(twF, static_cast<const cpx<R>*>(a.tw));
        __syncthreads();
    };
    // the product pass reads the table entries into registers ahead of its
    // data loads and writes them to LDS after issuing those (a fill issued
    // behind the data loads would wait for all of them)
    constexpr int NT = G * U;
    cpx<R> ti[PI::template tw_per_thread<NT> > 0 ? PI::template tw_per_thread<NT> : 1];
    cpx<R> tf[PF::template tw_per_thread<NT> > 0 ? PF::template tw_per_thread<NT> : 1];
    // (FP32 only: the FP64 build keeps the staged entries in scratch memory)
    constexpr bool STAGE = MODE == X_RHS && BPC == 0 && sizeof(R) == 4 && !WS;
    if constexpr (STAGE) {
        PI::template fetch_tw<NT>(ti, static_cast<const cpx<R>*>(a.tw));
        if constexpr (!SAME) PF::template fetch_tw<NT>(tf, static_cast<const cpx<R>*>(a.tw));
    } else {
        tables();
    }
    static_assert(BPC == 0 || MODE == X_RHS, "persistent blocks are for the product pass");
    const int tid = threadIdx.x, u = tid / G, t = tid % G, t0 = t;
    cpx<R>* my = reinterpret_cast<cpx<R>*>(smem_raw) + u * LL;
    long long samp = 0, l1 = 0;
    bool valid = false;
    auto set_tile = [&](long long tile) {
        const long long unit = tile * U + u;
        valid = unit < a.nunits;
        const long long L = valid ? 2 * unit : 0;
        samp = L / ((long long)N * N);
        l1 = L % ((long long)N * N);
    };
    if constexpr (BPC == 0) set_tile(xcd_tile(gridDim.x));
    constexpr int K = (N - 1) / 3, Mx = K + 1;

    // inverse (C2R) of component c of both lines into z = a + i b: the
    // Hermitian input of the packed transform, then the transform
    auto load_raw = [&](int c, cpx<R>(&v)[E]) {
        const cpx<R>* p1 = static_cast<const cpx<R>*>(a.in) + samp * a.in_ss + c * a.in_cs + l1 * Mx;
        const cpx<R>* p2 = p1 + Mx;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = PI::in_pos(t, i);
            cpx<R> A = {0, 0}, B = {0, 0};
            if (valid) {
                if (n <= K) {
                    A = p1[n];
                    B = p2[n];
                    if (n == 0) A.y = B.y = 0;
                } else if (n >= N - K) {
                    const cpx<R> a1 = p1[N - n], b1 = p2[N - n];
                    A = {a1.x, -a1.y};
                    B = {b1.x, -b1.y};
                }
            }
            v[i] = {A.x - B.y, A.y + B.x};
        }
    };
    auto load_inv = [&](int c, cpx<R>(&v)[E]) {
        load_raw(c, v);
        int t = t0;
        asm volatile("" : "+v"(t));
        PI::template run<+1, 1, 0, true, WS>(v, t, my, twI);
    };

    // forward (R2C) of v = a + i b; store k_x <= K of both lines as product p
    // (v already transformed with SKIP)
    auto fwd_store = [&](int p, cpx<R>(&v)[E], auto skip) {
        if constexpr (!decltype(skip)::value) PF::template run<-1, 1, 0, true, WS>(v, t, my, twF);
#pragma unroll
        for (int i = 0; i < E; ++i) my[PF::out_pos(t, i)] = v[i];
        lds_sync<WS>();
        const R h = (R)(0.5 * a.scale);
        cpx<R>* o1 = static_cast<cpx<R>*>(a.out) + samp * a.out_ss + p * a.out_cs + l1 * Mx;
        cpx<R>* o2 = o1 + Mx;
        for (int kx = t; kx <= K; kx += G) {
            const cpx<R> zk = my[kx];
            const cpx<R> zm = my[(N - kx) % N];
            if (valid) {
                o1[kx] = {(zk.x + zm.x) * h, (zk.y - zm.y) * h};
                o2[kx] = {(zk.y + zm.y) * h, (zm.x - zk.x) * h};
            }
        }
        lds_sync<WS>();
    };

    // SHT = 3: v holds Z[b + m G], m < E (b = mirror_order(t) for lines of
    // 128 threads, t otherwise); the lane holding bins G - b has
    // Z[N - b - m G] in slot E - 1 - m
    auto fwd_store_mir = [&](int p, const cpx<R>(&v)[E]) {
        static_assert(SHT != 3 || ((G == 128 || (G <= 64 && 64 % G == 0)) && PF::RL == E && N == E * G && K < 3 * G),
                      "register unpack: lines of 128 threads or inside one wavefront, last radix E");
        const int b = G == 128 ? mirror_order(t) : t;
        const int pg = (G - b) & (G - 1);  // butterfly with the mirrored bins
        const int pl = 4 * (G == 128 ? mirror_lane(pg) : (int)(threadIdx.x & 63) - t + pg);
        auto bp = [&](R x) {
            if constexpr (sizeof(R) == 4) {
                return __builtin_bit_cast(R, __builtin_amdgcn_ds_bpermute(pl, __builtin_bit_cast(int, x)));
            } else {
                const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
                const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(pl, (int)(unsigned)u);
                const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(pl, (int)(unsigned)(u >> 32));
                return __builtin_bit_cast(R, ((unsigned long long)hi << 32) | lo);
            }
        };
        cpx<R> pm[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) pm[m] = {bp(v[E - 1 - m].x), bp(v[E - 1 - m].y)};
        const R h = (R)(0.5 * a.scale);
        cpx<R>* o1 = static_cast<cpx<R>*>(a.out) + samp * a.out_ss + p * a.out_cs + l1 * Mx;
        cpx<R>* o2 = o1 + Mx;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int kx = b + m * G;
            const cpx<R> zk = v[m];
            const cpx<R> zm = b == 0 ? v[(E - m) % E] : pm[m];  // bin 0 mirrors onto its own thread
            if (valid && kx <= K) {
                o1[kx] = {(zk.x + zm.x) * h, (zk.y - zm.y) * h};
                o2[kx] = {(zk.y + zm.y) * h, (zm.x - zk.x) * h};
            }
        }
    };

    if constexpr (MODE == X_RHS) {
      auto body = [&] {
        cpx<R> z[3][E], v[E];
        // all three loads in flight before the first transform
        load_raw(0, z[0]);
        load_raw(1, z[1]);
        load_raw(2, z[2]);
        if constexpr (STAGE) {
            PI::template put_tw<NT>(twI, ti);
            if constexpr (!SAME) PF::template put_tw<NT>(twF, tf);
            __syncthreads();
        }
        if constexpr (SHT > 0) {
            PI::template run_n<+1, 1, 0, true, WS>(z, t, my, twI);
        } else {
            PI::template run<+1, 1, 0, true, WS>(z[0], t, my, twI);
            PI::template run<+1, 1, 0, true, WS>(z[1], t, my, twI);
            PI::template run<+1, 1, 0, true, WS>(z[2], t, my, twI);
        }
        // B_ij = u_i u_j, upper triangle (xx, xy, xz, yy, yz, zz); real parts
        // belong to line l1, imaginary parts to line l2
        auto mul = [&](cpx<R>(&o)[E], const cpx<R>(&za)[E], const cpx<R>(&zb)[E]) {
#pragma unroll
            for (int i = 0; i < E; ++i) o[i] = {za[i].x * zb[i].x, za[i].y * zb[i].y};
        };
        if constexpr (SHT == 3) {
            auto fwd = [&](auto& w) { PF::template run_n<-1, 1, 0, true, WS, G == 128>(w, t, my, twF); };
            {
                cpx<R> w[1][E];
                mul(w[0], z[0], z[0]);
                fwd(w);
                fwd_store_mir(0, w[0]);
            }
            {
                cpx<R> w[2][E];
                mul(w[0], z[0], z[1]);
                mul(w[1], z[0], z[2]);
                fwd(w);
                fwd_store_mir(1, w[0]);
                fwd_store_mir(2, w[1]);
            }
            {
                cpx<R> w[3][E];
                mul(w[0], z[1], z[1]);
                mul(w[1], z[1], z[2]);
                mul(w[2], z[2], z[2]);
                fwd(w);
                fwd_store_mir(3, w[0]);
                fwd_store_mir(4, w[1]);
                fwd_store_mir(5, w[2]);
            }
        } else if constexpr (SHT == 2) {
            using T_ = std::true_type;
            mul(v, z[0], z[0]);
            fwd_store(0, v, std::false_type{});
            {
                cpx<R> w[2][E];
                mul(w[0], z[0], z[1]);
                mul(w[1], z[0], z[2]);
                PF::template run_n<-1, 1, 0, true, WS>(w, t, my, twF);
                fwd_store(1, w[0], T_{});
                fwd_store(2, w[1], T_{});
            }
            {
                cpx<R> w[3][E];
                mul(w[0], z[1], z[1]);
                mul(w[1], z[1], z[2]);
                mul(w[2], z[2], z[2]);
                PF::template run_n<-1, 1, 0, true, WS>(w, t, my, twF);
                fwd_store(3, w[0], T_{});
                fwd_store(4, w[1], T_{});
                fwd_store(5, w[2], T_{});
            }
        } else {
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                switch (p) {
                    case 0: mul(v, z[0], z[0]); break;
                    case 1: mul(v, z[0], z[1]); break;
                    case 2: mul(v, z[0], z[2]); break;
                    case 3: mul(v, z[1], z[1]); break;
                    case 4: mul(v, z[1], z[2]); break;
                    default: mul(v, z[2], z[2]); break;
                }
                fwd_store(p, v, std::false_type{});
            }
        }
      };
      if constexpr (BPC > 0) {
          const long long ntiles = (a.nunits + U - 1) / U;
#pragma unroll 1
          for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
              set_tile(tile);
              body();
          }
      } else {
          body();
      }
    } else if constexpr (MODE == X_ADJ) {
        // inputs: components 0..4 the trace-free strain S (xx, xy, xz, yy,
        // yz), 5..7 the velocity; a_i = 2 sum_j S_ij u_j, upper triangle
        // (i, j) adds S_ij u_j to a_i and, off the diagonal, S_ij u_i to a_j;
        // S_zz = -S_xx - S_yy adds -2 (S_xx + S_yy) u_z to a_z.
        // With xadj_park: the transformed velocities wait in this line pair's
        // slice of LDS instead of registers; every thread reads back only the
        // elements it wrote (the strain comes out of the same plan at the
        // same positions), so no barrier is needed.
        constexpr bool PARK = xadj_park<PI, PF, U, R>();
        cpx<R> aa[3][E], v[E];
        cpx<R>(&a0)[E] = aa[0];
        cpx<R>(&a1)[E] = aa[1];
        cpx<R>(&a2)[E] = aa[2];
        cpx<R> ur[PARK ? 1 : 3][E];
        cpx<R>* uv = twI + (SAME ? PI::tw_len : PI::tw_len + PF::tw_len) + u * 3 * N;
        if constexpr (PARK) {
#pragma unroll 1
            for (int c = 0; c < 3; ++c) {
                load_inv(5 + c, v);
#pragma unroll
                for (int i = 0; i < E; ++i) uv[c * N + PI::out_pos(t, i)] = v[i];
            }
        } else {
            load_inv(5, ur[0]);
            load_inv(6, ur[1]);
            load_inv(7, ur[2]);
        }
#pragma unroll
        for (int i = 0; i < E; ++i) a0[i] = a1[i] = a2[i] = cpx<R>{0, 0};
        // acc += f S u_c
        auto fma2 = [&](cpx<R>(&acc)[E], const cpx<R>(&s)[E], int c, R f) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                cpx<R> w;
                if constexpr (PARK) w = uv[c * N + PI::out_pos(t, i)];
                else w = c == 0 ? ur[0][i] : (c == 1 ? ur[1][i] : ur[2][i]);
                acc[i].x += f * s[i].x * w.x;
                acc[i].y += f * s[i].y * w.y;
            }
        };
#pragma unroll 1
        for (int p = 0; p < 5; ++p) {
            load_inv(p, v);
            switch (p) {
                case 0: fma2(a0, v, 0, 2); fma2(a2, v, 2, -2); break;
                case 1: fma2(a0, v, 1, 2); fma2(a1, v, 0, 2); break;
                case 2: fma2(a0, v, 2, 2); fma2(a2, v, 0, 2); break;
                case 3: fma2(a1, v, 1, 2); fma2(a2, v, 2, -2); break;
                default: fma2(a1, v, 2, 2); fma2(a2, v, 1, 2); break;
            }
        }
        if constexpr (SHT >= 3) {
            // the three forward transforms grouped, then the register unpack
            PF::template run_n<-1, 1, 0, true, WS, G == 128>(aa, t, my, twF);
            fwd_store_mir(0, aa[0]);
            fwd_store_mir(1, aa[1]);
            fwd_store_mir(2, aa[2]);
        } else {
            fwd_store(0, a0, std::false_type{});
            fwd_store(1, a1, std::false_type{});
            fwd_store(2, a2, std::false_type{});
        }
    } else if constexpr (MODE == X_INV3) {
        cpx<R> v[E];
        for (int c = 0; c < 3; ++c) {
            load_inv(c, v);
            R* o1 = static_cast<R*>(a.out) + samp * a.out_ss + c * a.out_cs + l1 * N;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int x = PI::out_pos(t, i);
                if (valid) {
                    o1[x] = v[i].x;
                    o1[N + x] = v[i].y;
                }
            }
        }
    } else {  // X_FWD3
        cpx<R> v[E];
        for (int c = 0; c < 3; ++c) {
            const R* p1 = static_cast<const R*>(a.in) + samp * a.in_ss + c * a.in_cs + l1 * N;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int x = PF::in_pos(t, i);
                v[i] = valid ? cpx<R>{p1[x], p1[N + x]} : cpx<R>{0, 0};
            }
            fwd_store(c, v, std::false_type{});
        }
    }
}

// ------------------------------------------------------------------ X pass, half-length form
// Each real x-line of length N is transformed by a complex transform of
// length H = N/2 held by G <= 64 threads of one wavefront (the line's
// exchanges need no block barrier).  The C2R packs even and odd samples, z_m = x_{2m} + i x_{2m+1}:
// splitting x_n = sum_k X_k exp(2 pi i k n / N) by the parity of n and
// folding k + H onto k gives z = IDFT_H(Z) with
//   Z_k = (X_k + conj X_{H-k}) + i W^{-k} (X_k - conj X_{H-k}),  W = exp(-2 pi i / N),
// for k < H (X_{H-k} = 0 above the cutoff; the Nyquist mode X_H is truncated).
// The R2C of a real product line y unpacks Z = DFT_H(y_{2m} + i y_{2m+1}):
//   Y_k = (Z_k + conj Z_{H-k}) / 2 - (i / 2) W^k (Z_k - conj Z_{H-k}),  Z_H = Z_0,
// which are the even-sample and odd-sample transforms recombined.  A lane
// holds the same positions k = t + G i at the input and the output of the
// plan, so one register set of W^k serves both.
// SHT as for k_xline (2: inverse and forward transforms grouped).
template <class PH, int U, int W, typename R, int SHT = 0>
__global__ void __launch_bounds__(PH::G* U, W) k_xhalf(XArgs a)
{
    constexpr int H = PH::N, N = 2 * H, G = PH::G, E = PH::E;
    static_assert(G <= 64 && 64 % G == 0, "lines inside one wavefront");
    static_assert(PH::R0 == PH::RL, "the forward transform takes the inverse's output order");
    static_assert(PH::R0 == E, "a lane's positions are t + G i, i < E");
    constexpr int K = (N - 1) / 3, Mx = K + 1;
    static_assert(K < H, "the cutoff lies below the Nyquist mode");
    constexpr int LL = PH::template lds_len_st<sizeof(cpx<R>)>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* twl = reinterpret_cast<cpx<R>*>(smem_raw) + U * LL;
    PH::template fill_tw_from<2, R>(twl, static_cast<const cpx<R>*>(a.tw));
    const int tid = threadIdx.x, u = tid / G, t = tid % G;
    cpx<R>* my = reinterpret_cast<cpx<R>*>(smem_raw) + u * LL;
    const long long line = xcd_tile(gridDim.x) * U + u;
    const bool valid = line < 2 * a.nunits;
    const long long L = valid ? line : 0;
    const long long samp = L / ((long long)N * N), l1 = L % ((long long)N * N);
    const cpx<R>* __restrict__ tw = static_cast<const cpx<R>*>(a.tw);
    static_assert(PH::in_pos(1, 1) == PH::out_pos(1, 1), "input and output positions coincide");
    cpx<R> wk[E];  // W^k at this lane's positions
#pragma unroll
    for (int i = 0; i < E; ++i) wk[i] = tw[PH::in_pos(t, i)];
    __syncthreads();  // stage tables

    // Z of component c of this line, from its half spectrum
    auto load_z = [&](int c, cpx<R>(&z)[E]) {
        const cpx<R>* __restrict__ p = static_cast<const cpx<R>*>(a.in) + samp * a.in_ss + c * a.in_cs + l1 * Mx;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = PH::in_pos(t, i);
            cpx<R> A = {0, 0}, Bc = {0, 0};  // X_k and conj X_{H-k}
            if (valid) {
                if (k <= K) {
                    A = p[k];
                    if (k == 0) A.y = 0;  // the Hermitian part of the k = 0 mode
                }
                if (H - k <= K) {
                    const cpx<R> b = p[H - k];
                    Bc = {b.x, -b.y};
                }
            }
            const cpx<R> sm = {A.x + Bc.x, A.y + Bc.y}, d = {A.x - Bc.x, A.y - Bc.y};
            const cpx<R> e = {wk[i].x * d.x + wk[i].y * d.y, wk[i].x * d.y - wk[i].y * d.x};  // W^{-k} d
            z[i] = {sm.x - e.y, sm.y + e.x};
        }
    };
    // forward transform of the packed product v, then Y_k, k <= K, of product p
    auto fwd_store = [&](int p, cpx<R>(&v)[E], auto skip) {
        if constexpr (!decltype(skip)::value) PH::template run<-1, 1, 0, true, true>(v, t, my, twl);
#pragma unroll
        for (int i = 0; i < E; ++i) my[PH::out_pos(t, i)] = v[i];
        lds_sync<true>();
        const R h = (R)(0.5 * a.scale);
        cpx<R>* o = static_cast<cpx<R>*>(a.out) + samp * a.out_ss + p * a.out_cs + l1 * Mx;
#pragma unroll
        for (int j = 0; j * G <= K; ++j) {
            const int k = t + j * G;
            if (k <= K) {
                const cpx<R> zk = my[k], zm = my[(H - k) % H];
                const cpx<R> sm = {zk.x + zm.x, zk.y - zm.y}, d = {zk.x - zm.x, zk.y + zm.y};
                const cpx<R> f = {wk[j].x * d.x - wk[j].y * d.y, wk[j].x * d.y + wk[j].y * d.x};  // W^k d
                if (valid) o[k] = {(sm.x + f.y) * h, (sm.y - f.x) * h};
            }
        }
        lds_sync<true>();
    };
    static_assert(K < E * G, "the lane's W^k set covers the stored modes");

    cpx<R> z[3][E], v[E];
    load_z(0, z[0]);
    load_z(1, z[1]);
    load_z(2, z[2]);
    if constexpr (SHT > 0) {
        PH::template run_n<+1, 1, 0, true, true>(z, t, my, twl);
    } else {
        PH::template run<+1, 1, 0, true, true>(z[0], t, my, twl);
        PH::template run<+1, 1, 0, true, true>(z[1], t, my, twl);
        PH::template run<+1, 1, 0, true, true>(z[2], t, my, twl);
    }
    // B_ij = u_i u_j (xx, xy, xz, yy, yz, zz): real parts are the even
    // samples, imaginary parts the odd ones
    auto mul = [&](cpx<R>(&o)[E], const cpx<R>(&za)[E], const cpx<R>(&zb)[E]) {
#pragma unroll
        for (int i = 0; i < E; ++i) o[i] = {za[i].x * zb[i].x, za[i].y * zb[i].y};
    };
    if constexpr (SHT == 2) {
        using T_ = std::true_type;
        mul(v, z[0], z[0]);
        fwd_store(0, v, std::false_type{});
        {
            cpx<R> w[2][E];
            mul(w[0], z[0], z[1]);
            mul(w[1], z[0], z[2]);
            PH::template run_n<-1, 1, 0, true, true>(w, t, my, twl);
            fwd_store(1, w[0], T_{});
            fwd_store(2, w[1], T_{});
        }
        {
            cpx<R> w[3][E];
            mul(w[0], z[1], z[1]);
            mul(w[1], z[1], z[2]);
            mul(w[2], z[2], z[2]);
            PH::template run_n<-1, 1, 0, true, true>(w, t, my, twl);
            fwd_store(3, w[0], T_{});
            fwd_store(4, w[1], T_{});
            fwd_store(5, w[2], T_{});
        }
    } else {
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            switch (p) {
                case 0: mul(v, z[0], z[0]); break;
                case 1: mul(v, z[0], z[1]); break;
                case 2: mul(v, z[0], z[2]); break;
                case 3: mul(v, z[1], z[1]); break;
                case 4: mul(v, z[1], z[2]); break;
                default: mul(v, z[2], z[2]); break;
            }
            fwd_store(p, v, std::false_type{});
        }
    }
}

// ------------------------------------------------------------------ F3 pass
// PRE = 1 issues the loads of component p + 1 before the transform of p.
// ZI = 1 (F3_RHS only) also transforms the new state back along z, zero-
// padded to N rows, and writes it to a.zinv: the inverse z pass of the next
// stage's right-hand side, done while the state is still in registers.
// DB = 1 double-buffers the LDS exchanges (one barrier per exchange).
template <class P, int T, int MODE, int SP, int W, typename R, int PRE = 0, int ZI = 0, int DB = 0>
__global__ void __launch_bounds__(P::G* T, W) k_f3(F3Args a)
{
    constexpr int N = P::N, E = P::E;
    constexpr int NC = MODE == F3_RHS ? 6 : 3;  // F3_PROJ and F3_ADJ take 3 components
    static_assert(ZI == 0 || MODE == F3_RHS, "the fused inverse follows the stage epilogue");
    static_assert(P::slot_map_ok(), "output and input slots of a thread cover the same rows");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TB = (int)tile_bytes<P, T, SP, R>();
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* twl = reinterpret_cast<cpx<R>*>(smem_raw + (DB ? 2 : 1) * TB);
    P::template load_tw<R>(twl, static_cast<const cpx<R>*>(a.tw));
    int par = 0;  // next exchange buffer (DB)
    // transform of v in direction D by the tile's LDS (column cc)
    auto fft = [&](auto dir, cpx<R>(&v)[E], int gg, int cc) {
        constexpr int D = decltype(dir)::value;
        cpx<R>* base = SP ? reinterpret_cast<cpx<R>*>(reinterpret_cast<R*>(lds) + cc) : lds + cc;
        if constexpr (DB) P::template run_db<D, T, SP>(v, gg, base, twl, TB, par);
        else P::template run<D, T, SP>(v, gg, base, twl);
    };
    const int tid = threadIdx.x, c = tid % T, g = tid / T;
    constexpr int K = Cut<N>::K, M = Cut<N>::M, Mx = K + 1;
    // column of this thread in tile `tile`
    struct Col {
        bool valid;
        long long samp;
        int s;
    };
    constexpr int CB = compact_cb(sizeof(cpx<R>));
    const long long cols = compact_cols(a.MMx, sizeof(cpx<R>));  // padded columns per sample
    auto column = [&](long long tile) {
        const long long q = tile * T + c;
        Col k;
        k.valid = q < a.Q && q % cols < a.MMx;
        k.samp = k.valid ? q / cols : 0;
        k.s = k.valid ? (int)(q % cols) : 0;
        return k;
    };
    auto load = [&](int p, cpx<R>(&v)[E], int gg, const Col& k) {
        const cpx<R>* __restrict__ in = static_cast<const cpx<R>*>(a.in) + k.samp * a.in_ss + k.s;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = P::in_pos(gg, i);
            v[i] = k.valid ? in[p * a.in_cs + (long long)n * a.MMx] : cpx<R>{0, 0};
        }
    };
    cpx<R> nxt[PRE ? E : 1];
    // the tile: the component loop, then the epilogue (and the fused inverse)
    auto tile_body = [&](const Col& col) {
    const bool valid = col.valid;
    const long long samp = col.samp;
    const int s = col.s;
    const int jy = s / Mx, kxi = s % Mx;
    const int kyi = jy <= K ? jy : jy - M;
    const R kx = (R)kxi, ky = (R)kyi;

    cpx<R> acc[3][E];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < E; ++i) acc[j][i] = {0, 0};

    // transform of component p (in v) and its accumulation
    auto component = [&](int p, cpx<R>(&v)[E], int gg, int cc) {
        fft(std::integral_constant<int, -1>{}, v, gg, cc);
        if constexpr (MODE == F3_RHS) {
            // component p = (i, j) of the upper triangle adds k_j B to b_i
            // and, off the diagonal, k_i B to b_j: b_r += (wxy_r + wz_r k_z) B
            R w[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // [r][axis]
            switch (p) {
                case 0: w[0][0] = 1; break;
                case 1: w[0][1] = 1; w[1][0] = 1; break;
                case 2: w[0][2] = 1; w[2][0] = 1; break;
                case 3: w[1][1] = 1; break;
                case 4: w[1][2] = 1; w[2][1] = 1; break;
                default: w[2][2] = 1; break;
            }
            const R wxy0 = w[0][0] * kx + w[0][1] * ky, wz0 = w[0][2];
            const R wxy1 = w[1][0] * kx + w[1][1] * ky, wz1 = w[1][2];
            const R wxy2 = w[2][0] * kx + w[2][1] * ky, wz2 = w[2][2];
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int n = P::out_pos(g, i);
                const R kz = (R)(n < N / 2 ? n : n - N);
                const R c0 = wxy0 + wz0 * kz, c1 = wxy1 + wz1 * kz, c2 = wxy2 + wz2 * kz;
                acc[0][i].x += c0 * v[i].x;
                acc[0][i].y += c0 * v[i].y;
                acc[1][i].x += c1 * v[i].x;
                acc[1][i].y += c1 * v[i].y;
                acc[2][i].x += c2 * v[i].x;
                acc[2][i].y += c2 * v[i].y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                acc[0][i] = p == 0 ? v[i] : acc[0][i];
                acc[1][i] = p == 1 ? v[i] : acc[1][i];
                acc[2][i] = p == 2 ? v[i] : acc[2][i];
            }
        }
    };

    {
        // the three-component modes unroll the loop: a runtime component index
        // would turn the assignment into acc[p] and push acc to scratch memory
        constexpr int UNR = MODE == F3_RHS ? 1 : NC;
#pragma unroll UNR
        for (int p = 0; p < NC; ++p) {
            // opaque copies of the thread coordinates: the addresses derived
            // from them are recomputed per component instead of being hoisted
            // out of the loop, which would hold them in registers throughout
            int gg = g, cc = c;
            asm volatile("" : "+v"(gg), "+v"(cc));
            cpx<R> v[E];
            if constexpr (PRE) {
#pragma unroll
                for (int i = 0; i < E; ++i) v[i] = nxt[i];
                if (p + 1 < NC) load(p + 1, nxt, gg, col);
            } else {
                load(p, v, gg, col);
            }
            component(p, v, gg, cc);
        }
    }

    const R sc = (R)a.scale;
    const double dts = (MODE != F3_PROJ && valid) ? a.dt[samp] : 0.0;
    const R* __restrict__ rate = static_cast<const R*>(a.rate);

    // Epilogue.  The state reads of a group of output slots are all issued
    // before any of the group's arithmetic and stores, so their latencies
    // overlap (the output may alias a state that is read, so loads cannot be
    // moved across earlier stores).  Slots that hold a truncated row for
    // every thread are skipped at compile time.
    // row kz of slot i and its compact index (-1: truncated)
    auto row = [&](int i, int& kzi, int& jz) {
        const int n = P::out_pos(g, i);
        jz = valid ? compact_of(n, N, K, M) : -1;
        kzi = n <= K ? n : n - N;
    };
    // -i sum_j k_j B_ij (or the transform itself), scaled, then the Leray
    // projection (not for the adjoint, which acts on the whole cube)
    auto contracted = [&](int i, int kzi, cpx<R>(&b)[3]) {
        const R kz = (R)kzi;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if constexpr (MODE == F3_RHS) b[j] = {acc[j][i].y * sc, -acc[j][i].x * sc};  // -i * sum
            else b[j] = {acc[j][i].x * sc, acc[j][i].y * sc};
        }
        if constexpr (MODE == F3_ADJ) return;
        const int k2 = kxi * kxi + kyi * kyi + kzi * kzi;
        if (k2 > 0) {
            const R inv = (R)1 / (R)k2;
            const cpx<R> kb = {kx * b[0].x + ky * b[1].x + kz * b[2].x, kx * b[0].y + ky * b[1].y + kz * b[2].y};
            const R kv[3] = {kx, ky, kz};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                b[j].x -= kv[j] * kb.x * inv;
                b[j].y -= kv[j] * kb.y * inv;
            }
        }
    };
    // compact offset of row jz of component 0 (components are st_cs apart)
    auto st_of = [&](int jz) {
        return samp * a.st_ss + (long long)((unsigned)s / CB) * 3 * a.st_cs + (long long)jz * CB + (unsigned)s % CB;
    };
    auto k2_of = [&](int kzi) { return kxi * kxi + kyi * kyi + kzi * kzi; };

    if constexpr (MODE == F3_PROJ) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            if (!slot_may_keep<P>(i)) continue;
            int kzi, jz;
            row(i, kzi, jz);
            if (jz < 0) continue;
            cpx<R> b[3];
            contracted(i, kzi, b);
            cpx<R>* o = static_cast<cpx<R>*>(a.out) + st_of(jz);
#pragma unroll
            for (int j = 0; j < 3; ++j) o[j * a.st_cs] = b[j];
        }
    } else if constexpr (MODE == F3_RHS) {
        // out = ca u0 + cb us + cc dt F, F = c - rate us; u0 is read only when
        // ca != 0 (uniform over the launch)
        auto epilogue = [&](auto with_u0) {
            constexpr bool U0 = decltype(with_u0)::value;
            const R ca = (R)a.ca, cb = (R)a.cb, cdt = (R)(a.cc * dts);
            const cpx<R>* __restrict__ us = static_cast<const cpx<R>*>(a.us);
            const cpx<R>* __restrict__ u0 = static_cast<const cpx<R>*>(a.u0);
            cpx<R>* o = static_cast<cpx<R>*>(a.out);
            constexpr int GS = U0 ? E / 2 : E;  // slots per load group (registers)
#pragma unroll
            for (int i0 = 0; i0 < E; i0 += GS) {
                cpx<R> w[GS][3], w0[U0 ? GS : 1][3];
                R rt[GS];
#pragma unroll
                for (int d = 0; d < GS; ++d) {
                    const int i = i0 + d;
                    if (i >= E || !slot_may_keep<P>(i)) continue;
                    int kzi, jz;
                    row(i, kzi, jz);
                    if (jz < 0) continue;
                    const long long st = st_of(jz);
                    rt[d] = rate[k2_of(kzi)];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        w[d][j] = us[st + j * a.st_cs];
                        if constexpr (U0) w0[d][j] = u0[st + j * a.st_cs];
                    }
                }
#pragma unroll
                for (int d = 0; d < GS; ++d) {
                    const int i = i0 + d;
                    if (i >= E) continue;
                    if (!slot_may_keep<P>(i)) {
                        if constexpr (ZI) {  // truncated rows enter the inverse as zeros
#pragma unroll
                            for (int j = 0; j < 3; ++j) acc[j][i] = {0, 0};
                        }
                        continue;
                    }
                    int kzi, jz;
                    row(i, kzi, jz);
                    if (jz < 0) {
                        if constexpr (ZI) {
#pragma unroll
                            for (int j = 0; j < 3; ++j) acc[j][i] = {0, 0};
                        }
                        continue;
                    }
                    cpx<R> b[3];
                    contracted(i, kzi, b);
                    const long long st = st_of(jz);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const cpx<R> ww = w[d][j];
                        cpx<R> f = {b[j].x - rt[d] * ww.x, b[j].y - rt[d] * ww.y};
                        cpx<R> r = {cb * ww.x + cdt * f.x, cb * ww.y + cdt * f.y};
                        if constexpr (U0) {
                            r.x += ca * w0[d][j].x;
                            r.y += ca * w0[d][j].y;
                        }
                        o[st + j * a.st_cs] = r;
                        if constexpr (ZI) acc[j][i] = r;
                    }
                }
            }
        };
        if (a.ca != 0.0) epilogue(std::true_type{});
        else epilogue(std::false_type{});
    } else {  // F3_ADJ
        // out = ca L3 + c2 L2 + c1 L1 + cc dt (T a - rate lam), no projection;
        // L3 = u0, lam = us.  A term with a zero coefficient is not read, and
        // L1 is not read again when it is lam itself.
        auto epilogue = [&](auto with3, auto with2, auto with1) {
            constexpr bool H3 = decltype(with3)::value, H2 = decltype(with2)::value, H1 = decltype(with1)::value;
            const R c3 = (R)a.ca, c2 = (R)a.c2, c1 = (R)a.c1, cdt = (R)(a.cc * dts);
            const bool l1_is_lam = a.l1 == a.us;
            const cpx<R>* __restrict__ lam = static_cast<const cpx<R>*>(a.us);
            const cpx<R>* __restrict__ L3 = static_cast<const cpx<R>*>(a.u0);
            const cpx<R>* __restrict__ L2 = static_cast<const cpx<R>*>(a.l2);
            const cpx<R>* __restrict__ L1 = static_cast<const cpx<R>*>(H1 ? (l1_is_lam ? a.us : a.l1) : a.us);
            cpx<R>* o = static_cast<cpx<R>*>(a.out);
            constexpr int NL = 1 + H3 + H2 + H1;
            constexpr int GS = NL <= 1 ? E : (NL == 2 ? E / 2 : E / 4 > 0 ? E / 4 : 1);
#pragma unroll
            for (int i0 = 0; i0 < E; i0 += GS) {
                cpx<R> wl[GS][3], w3[H3 ? GS : 1][3], w2[H2 ? GS : 1][3], w1[H1 ? GS : 1][3];
                R rt[GS];
#pragma unroll
                for (int d = 0; d < GS; ++d) {
                    const int i = i0 + d;
                    if (i >= E || !slot_may_keep<P>(i)) continue;
                    int kzi, jz;
                    row(i, kzi, jz);
                    if (jz < 0) continue;
                    const long long st = st_of(jz);
                    rt[d] = rate[k2_of(kzi)];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        wl[d][j] = lam[st + j * a.st_cs];
                        if constexpr (H3) w3[d][j] = L3[st + j * a.st_cs];
                        if constexpr (H2) w2[d][j] = L2[st + j * a.st_cs];
                        if constexpr (H1) {
                            if (!l1_is_lam) w1[d][j] = L1[st + j * a.st_cs];
                        }
                    }
                }
#pragma unroll
                for (int d = 0; d < GS; ++d) {
                    const int i = i0 + d;
                    if (i >= E || !slot_may_keep<P>(i)) continue;
                    int kzi, jz;
                    row(i, kzi, jz);
                    if (jz < 0) continue;
                    cpx<R> b[3];
                    contracted(i, kzi, b);
                    const long long st = st_of(jz);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const cpx<R> w = wl[d][j];
                        cpx<R> r = {cdt * (b[j].x - rt[d] * w.x), cdt * (b[j].y - rt[d] * w.y)};
                        if constexpr (H3) {
                            r.x += c3 * w3[d][j].x;
                            r.y += c3 * w3[d][j].y;
                        }
                        if constexpr (H2) {
                            r.x += c2 * w2[d][j].x;
                            r.y += c2 * w2[d][j].y;
                        }
                        if constexpr (H1) {
                            const cpx<R> z = l1_is_lam ? w : w1[d][j];
                            r.x += c1 * z.x;
                            r.y += c1 * z.y;
                        }
                        o[st + j * a.st_cs] = r;
                    }
                }
            }
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        const bool h3 = a.ca != 0.0, h2 = a.c2 != 0.0, h1 = a.c1 != 0.0;
        if (h3 && !h2 && !h1) epilogue(T_{}, F_{}, F_{});
        else if (!h3 && h2 && !h1) epilogue(F_{}, T_{}, F_{});
        else if (h3 && h2 && h1) epilogue(T_{}, T_{}, T_{});
        else if (h3 && h2) epilogue(T_{}, T_{}, F_{});
        else if (h3 && h1) epilogue(T_{}, F_{}, T_{});
        else if (h2 && h1) epilogue(F_{}, T_{}, T_{});
        else if (h1) epilogue(F_{}, F_{}, T_{});
        else epilogue(F_{}, F_{}, F_{});
    }
    if constexpr (ZI) {
        // acc[j][i] holds row out_pos(g, i) of component j of the new state
        // (zero outside the retained rows); slot i of the inverse input is
        // row in_pos(g, i) = out_pos(g, out_slot_of_in(i)).  One rolled loop
        // over the components keeps a single copy of the transform; it always
        // takes acc[0] and shifts the others down (constant indices only: a
        // component-indexed read would move acc to scratch memory).
        cpx<R>* zo = static_cast<cpx<R>*>(a.zinv) + samp * a.in_ss + s;
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            int gg = g, cc = c;
            asm volatile("" : "+v"(gg), "+v"(cc));
            cpx<R> v[E];
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = acc[0][P::out_slot_of_in(i)];
#pragma unroll
            for (int i = 0; i < E; ++i) {
                acc[0][i] = acc[1][i];
                acc[1][i] = acc[2][i];
            }
            fft(std::integral_constant<int, +1>{}, v, gg, cc);
            if (valid) {
#pragma unroll
                for (int i = 0; i < E; ++i) zo[j * a.in_cs + (long long)P::out_pos(gg, i) * a.MMx] = v[i];
            }
        }
    }
    };  // tile_body

    const Col col = column(xcd_tile(gridDim.x));
    if constexpr (PRE) load(0, nxt, g, col);
    tile_body(col);
}

// ------------------------------------------------------------ adjoint z pass
// The first pass of the adjoint's vector-Jacobian product: per tile of T
// compact columns, lam and u are read once (three components each, the
// retained rows), mu = P lam is formed in registers, and the five stored
// components (xx, xy, xz, yy, yz) of the trace-free strain
// S_ab = (i/2)(k_a mu_b + k_b mu_a) and the three of u are each transformed
// back along z, zero-padded to N rows.  (The strain never goes to memory.)
template <class P, int T, int SP, int W, typename R>
__global__ void __launch_bounds__(P::G* T, W) k_strain_z(StrainZArgs a)
{
    constexpr int N = P::N, E = P::E;
    constexpr int K = Cut<N>::K, M = Cut<N>::M, Mx = K + 1;
    constexpr int CB = compact_cb(sizeof(cpx<R>));
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TB = (int)tile_bytes<P, T, SP, R>();
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* twl = reinterpret_cast<cpx<R>*>(smem_raw + TB);
    const int tid = threadIdx.x, c = tid % T, g = tid / T;
    const long long cols = compact_cols(a.MMx, sizeof(cpx<R>));
    const long long q = xcd_tile(gridDim.x) * T + c;
    const bool valid = q < a.Q && q % cols < a.MMx;
    const long long samp = valid ? q / cols : 0;
    const int s = valid ? (int)(q % cols) : 0;
    // compact offset of (component 0, row 0) of this column
    const long long st0 = samp * a.st_ss + (long long)((unsigned)s / CB) * 3 * a.st_cs + (unsigned)s % CB;
    auto load3 = [&](const void* src, cpx<R>(&v)[3][E]) {
        const cpx<R>* __restrict__ p = static_cast<const cpx<R>*>(src) + st0;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int jz = compact_of(P::in_pos(g, i), N, K, M);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                v[j][i] = (valid && jz >= 0) ? p[j * a.st_cs + (long long)jz * CB] : cpx<R>{0, 0};
        }
    };
    cpx<R> mu[3][E];
    load3(a.lam, mu);
    P::template load_tw<R>(twl, static_cast<const cpx<R>*>(a.tw));
    const int jy = s / Mx, kxi = s % Mx;
    const R kx = (R)kxi, ky = (R)(jy <= K ? jy : jy - M);
    // mu = P lam, mode by mode
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int n = P::in_pos(g, i);
        const R kz = (R)(n < N / 2 ? n : n - N);
        const R k2 = kx * kx + ky * ky + kz * kz;
        if (k2 > 0) {
            const R inv = (R)1 / k2;
            const R dx = (kx * mu[0][i].x + ky * mu[1][i].x + kz * mu[2][i].x) * inv;
            const R dy = (kx * mu[0][i].y + ky * mu[1][i].y + kz * mu[2][i].y) * inv;
            mu[0][i] = {mu[0][i].x - kx * dx, mu[0][i].y - kx * dy};
            mu[1][i] = {mu[1][i].x - ky * dx, mu[1][i].y - ky * dy};
            mu[2][i] = {mu[2][i].x - kz * dx, mu[2][i].y - kz * dy};
        }
    }
    auto transform_store = [&](int comp, cpx<R>(&v)[E]) {
        int gg = g, cc = c;
        asm volatile("" : "+v"(gg), "+v"(cc));
        cpx<R>* base = SP ? reinterpret_cast<cpx<R>*>(reinterpret_cast<R*>(lds) + cc) : lds + cc;
        P::template run<+1, T, SP>(v, gg, base, twl);
        cpx<R>* o = static_cast<cpx<R>*>(a.out) + samp * a.out_ss + comp * a.out_cs + s;
        if (valid) {
#pragma unroll
            for (int i = 0; i < E; ++i) o[(long long)P::out_pos(gg, i) * a.MMx] = v[i];
        }
    };
    // unrolled: a runtime component index would put mu in scratch memory
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        // the pair (a, b) of strain component p: xx, xy, xz, yy, yz
        const int ia = p < 3 ? 0 : 1, ib = p < 3 ? p : p - 2;
        cpx<R> v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = P::in_pos(g, i);
            const R kz = (R)(n < N / 2 ? n : n - N);
            const R ka = ia == 0 ? kx : ky;
            const R kb = ib == 0 ? kx : (ib == 1 ? ky : kz);
            const cpx<R> ma = ia == 0 ? mu[0][i] : mu[1][i];
            const cpx<R> mb = ib == 0 ? mu[0][i] : (ib == 1 ? mu[1][i] : mu[2][i]);
            const R wx = ka * mb.x + kb * ma.x, wy = ka * mb.y + kb * ma.y;
            v[i] = {(R)-0.5 * wy, (R)0.5 * wx};  // (i/2) w
        }
        transform_store(p, v);
    }
    cpx<R> uv[3][E];
    load3(a.u, uv);
    transform_store(5, uv[0]);
    transform_store(6, uv[1]);
    transform_store(7, uv[2]);
}

// ------------------------------------------------------------------ launch
template <typename Args>
inline hipError_t launch_k(void (*k)(Args), long long blocks, int threads, size_t lds, hipStream_t s, const Args& a,
                           bool& attr_done)
{
    if (blocks <= 0) return hipSuccess;
    if (lds > 65536 && !attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// the cutoff arguments must be the ones the kernels assume for length N
template <int N>
inline bool cut_ok(int K, int M)
{
    return K == Cut<N>::K && M == Cut<N>::M;
}

// Launchers of one schedule each.  W is the minimum number of waves per
// SIMD the compiler must allow (it caps the registers per thread).
template <class P, int T, int DIR, int MODE, int SP, int W, typename R, int DB = 0>
hipError_t launch_col(const ColArgs& a, hipStream_t s)
{
    constexpr size_t lds = (DB ? 2 : 1) * tile_bytes<P, T, SP, R>() + sizeof(cpx<R>) * P::tw_len;
    static_assert(P::G * T <= 1024, "at most 1024 threads per block");
    static_assert(lds <= 163840, "LDS per block exceeds 160 KiB");
    static bool done = false;
    if (!cut_ok<P::N>(a.K, a.M)) return hipErrorInvalidValue;
    return launch_k(k_colfft<P, T, DIR, MODE, SP, W, R, DB>, (a.Q + T - 1) / T, P::G * T, lds, s, a, done);
}

inline int device_cus()
{
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    }
    return n;
}

// persistent column pass with BPC resident blocks per compute unit
template <class P, int T, int DIR, int MODE, int SP, int W, int BPC, typename R>
hipError_t launch_col_p(const ColArgs& a, hipStream_t s)
{
    static_assert(P::G * T <= 1024, "at most 1024 threads per block");
    static_assert(tile_bytes<P, T, SP, R>() + sizeof(cpx<R>) * P::tw_len <= 163840, "LDS per block exceeds 160 KiB");
    static bool done = false;
    if (!cut_ok<P::N>(a.K, a.M)) return hipErrorInvalidValue;
    const long long ntiles = (a.Q + T - 1) / T;
    long long grid = (long long)device_cus() * BPC;
    if (grid > ntiles) grid = ntiles;
    return launch_k(k_colfft_p<P, T, DIR, MODE, SP, W, R>, grid, P::G * T,
                    tile_bytes<P, T, SP, R>() + sizeof(cpx<R>) * P::tw_len, s, a, done);
}

template <class PI, class PF, int U, int MODE, int W, typename R, int BPC = 0, bool WS = false, int SHT = 0>
hipError_t launch_x(const XArgs& a, hipStream_t s)
{
    constexpr int XL = x_line_len<PI, PF, R>();
    static_assert(PI::G * U <= 1024, "at most 1024 threads per block");
    constexpr int TW = std::is_same<PI, PF>::value ? PI::tw_len : PI::tw_len + PF::tw_len;
    constexpr int PK = MODE == X_ADJ && xadj_park<PI, PF, U, R>() ? 3 * PI::N * U : 0;  // parked velocities
    static_assert(sizeof(cpx<R>) * (XL * U + TW + PK) <= 163840, "LDS per block exceeds 160 KiB");
    static bool done = false;
    if (a.K != Cut<PI::N>::K) return hipErrorInvalidValue;
    long long grid = (a.nunits + U - 1) / U;
    if (BPC > 0 && grid > (long long)device_cus() * BPC) grid = (long long)device_cus() * BPC;
    return launch_k(k_xline<PI, PF, U, MODE, W, R, BPC, WS, SHT>, grid, PI::G * U,
                    sizeof(cpx<R>) * (XL * U + TW + PK), s, a, done);
}

// x pass in the half-length form: a.nunits pairs of lines, i.e. 2 a.nunits lines
template <class PH, int U, int W, typename R, int SHT = 0>
hipError_t launch_xh(const XArgs& a, hipStream_t s)
{
    constexpr int LL = PH::template lds_len_st<sizeof(cpx<R>)>();
    constexpr size_t lds = sizeof(cpx<R>) * ((size_t)LL * U + PH::tw_len);
    static_assert(PH::G * U <= 1024, "at most 1024 threads per block");
    static_assert(lds <= 163840, "LDS per block exceeds 160 KiB");
    static bool done = false;
    if (a.K != (2 * PH::N - 1) / 3) return hipErrorInvalidValue;
    return launch_k(k_xhalf<PH, U, W, R, SHT>, (2 * a.nunits + U - 1) / U, PH::G * U, lds, s, a, done);
}

template <class P, int T, int MODE, int SP, int W, typename R, int PRE = 0, int ZI = 0, int DB = 0>
hipError_t launch_f3(const F3Args& a, hipStream_t s)
{
    constexpr size_t lds = (DB ? 2 : 1) * tile_bytes<P, T, SP, R>() + sizeof(cpx<R>) * P::tw_len;
    static_assert(P::G * T <= 1024, "at most 1024 threads per block");
    static_assert(lds <= 163840, "LDS per block exceeds 160 KiB");
    static bool done = false;
    if (!cut_ok<P::N>(a.K, a.M) || a.Mx != Cut<P::N>::K + 1) return hipErrorInvalidValue;
    if (ZI && !a.zinv) return hipErrorInvalidValue;
    return launch_k(k_f3<P, T, MODE, SP, W, R, PRE, ZI, DB>, (a.Q + T - 1) / T, P::G * T, lds, s, a, done);
}

template <class P, int T, int SP, int W, typename R>
hipError_t launch_strain_z(const StrainZArgs& a, hipStream_t s)
{
    constexpr size_t lds = tile_bytes<P, T, SP, R>() + sizeof(cpx<R>) * P::tw_len;
    static_assert(P::G * T <= 1024, "at most 1024 threads per block");
    static_assert(lds <= 163840, "LDS per block exceeds 160 KiB");
    static bool done = false;
    if (!cut_ok<P::N>(a.K, a.M) || a.Mx != Cut<P::N>::K + 1) return hipErrorInvalidValue;
    return launch_k(k_strain_z<P, T, SP, W, R>, (a.Q + T - 1) / T, P::G * T, lds, s, a, done);
}

template <class V, class F>
inline void add_variant(V* list, int& n, F fn, const char* name)
{
    if (n < NS_MAXV) list[n++] = V{fn, name};
}

// Per-size default schedule: each pass has its own line plan (threads per
// line and radix order): the column passes (G, Rad), the x pass (GX, XRad
// and its reverse XRadRev for the forward half) and the fused z pass (GF,
// FRad); T / TF columns per block for the column and fused z passes and U
// line pairs per block for the x pass, for FP32 and FP64.  Sizes that are
// tuned add further variants in their translation unit.
template <int N>
struct SizeCfg;

template <int N, typename R>
struct Launch {
    using C = SizeCfg<N>;
    using P = Plan<N, C::G, typename C::Rad>;
    using PX = Plan<N, C::GX, typename C::XRad>;
    using PXR = Plan<N, C::GX, typename C::XRadRev>;
    using PF = Plan<N, C::GF, typename C::FRad>;
    static constexpr bool f64 = sizeof(R) == 8;
    static constexpr int T = f64 ? C::T64 : C::T32;
    static constexpr int TF = f64 ? C::TF64 : C::TF32;
    static constexpr int U = f64 ? C::U64 : C::U32;
    static constexpr int SP = f64 ? C::SP64 : C::SP32;
    static constexpr int SPF = f64 ? C::SPF64 : C::SPF32;

    static SizeKernels make()
    {
        SizeKernels k{};
        k.N = N;
        add_variant(k.inv, k.n_inv, launch_col<P, T, +1, COL_INV_PAD, SP, 1, R>, "default");
        add_variant(k.fwd, k.n_fwd, launch_col<P, T, -1, COL_FWD_TRUNC, SP, 1, R>, "default");
        add_variant(k.x, k.n_x, launch_x<PX, PXR, U, X_RHS, 1, R>, "default");
        add_variant(k.f3, k.n_f3, launch_f3<PF, TF, F3_RHS, SPF, 1, R>, "default");
        k.f3[k.n_f3 - 1].fn_zi = launch_f3<PF, TF, F3_RHS, SPF, 1, R, 0, 1>;
        k.x_fwd3 = launch_x<PX, PXR, U, X_FWD3, 1, R>;
        k.x_inv3 = launch_x<PX, PXR, U, X_INV3, 1, R>;
        k.f3_proj = launch_f3<PF, TF, F3_PROJ, SPF, 1, R>;
        k.strain_z = launch_strain_z<PF, TF, SPF, 1, R>;
        k.x_adj = launch_x<PX, PXR, U, X_ADJ, 1, R>;
        k.f3_adj = launch_f3<PF, TF, F3_ADJ, SPF, 1, R>;
        k.desc = C::desc;
        return k;
    }
};

}  // namespace ns
