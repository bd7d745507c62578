// Device FFT engine for gfx950: small-radix DFT codelets and a register
// Stockham (self-sorting, mixed-radix) FFT executed cooperatively by G
// threads per line, with the stages exchanged through LDS.
//
// A transform of length N with radices R_0..R_{S-1} (N = prod R_s) keeps
// E = N/G elements per thread in registers.  Before stage s (span
// P_s = R_0...R_{s-1}) thread t holds, for each of its butterflies
// b = t + q*G (q < N/(R_s G)), the inputs x[b + m N/R_s] (m < R_s) in
// v[q R_s + m].  The stage multiplies input m by w_{P_s R_s}^{m (b mod P_s)},
// applies a radix-R_s DFT and sends output m to position
// ((b - k) R_s + k) + m P_s, k = b mod P_s (Stockham autosort order).  After
// the last stage thread t holds X[t + q G + m N/R_last] in v[q R_last + m],
// i.e. outputs are in natural order with no bit reversal.  Twiddles come from
// a table exp(-2 pi i e / N) rounded from extended precision on the host,
// regrouped per stage in LDS (TwTable); the inverse direction uses the
// conjugate.
#pragma once
#include <hip/hip_runtime.h>

namespace ns {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * (DIR * i)
template <int DIR, typename R>
__device__ __forceinline__ cpx<R> mul_i(cpx<R> a)
{
    if constexpr (DIR > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
}
// a * w for DIR = -1, a * conj(w) for DIR = +1 (w from the forward table)
template <int DIR, typename R>
__device__ __forceinline__ cpx<R> twiddle(cpx<R> a, cpx<R> w)
{
    if constexpr (DIR < 0) return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
    else return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

// cos and sin of 2 pi j / 16
constexpr double kC16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                        0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                        -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                                        0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
constexpr double kS16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                        1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                        0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                        -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// cos and sin of 2 pi j / 12 (sqrt(3)/2 and 1/2 up to sign)
constexpr double kC12[12] = {1.0, 0.86602540378443864676, 0.5, 0.0, -0.5, -0.86602540378443864676,
                             -1.0, -0.86602540378443864676, -0.5, 0.0, 0.5, 0.86602540378443864676};
constexpr double kS12[12] = {0.0, 0.5, 0.86602540378443864676, 1.0, 0.86602540378443864676, 0.5,
                             0.0, -0.5, -0.86602540378443864676, -1.0, -0.86602540378443864676, -0.5};

// a * exp(DIR 2 pi i e / RR) for a compile-time exponent, RR dividing 16 or 12
template <int RR, int E, int DIR, typename R>
__device__ __forceinline__ cpx<R> rot_const(cpx<R> a)
{
    static_assert(16 % RR == 0 || 12 % RR == 0, "constant rotations for orders dividing 16 or 12");
    constexpr int e = E % RR;
    if constexpr (e == 0) return a;
    else if constexpr (4 * e == RR) return mul_i<DIR>(a);
    else if constexpr (2 * e == RR) return {-a.x, -a.y};
    else if constexpr (4 * e == 3 * RR) return mul_i<-DIR>(a);
    else if constexpr (16 % RR == 0) {
        constexpr int j = e * (16 / RR);
        const R c = (R)kC16[j];
        const R s = (R)(DIR * kS16[j]);
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    } else {
        constexpr int j = e * (12 / RR);
        const R c = (R)kC12[j];
        const R s = (R)(DIR * kS12[j]);
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// ---------------------------------------------------------------- codelets
// In-place y[k] = sum_m v[m] exp(DIR 2 pi i m k / R).
template <int R, int DIR, typename T>
struct Dft;

template <int DIR, typename T>
struct Dft<1, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>*) {}
};

template <int DIR, typename T>
struct Dft<2, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v)
    {
        cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int DIR, typename T>
struct Dft<3, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v)
    {
        const T s3 = (T)0.86602540378443864676;  // sin(2 pi / 3)
        cpx<T> a = v[0], b = v[1], c = v[2];
        cpx<T> t1 = cadd(b, c);
        cpx<T> t2 = {a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
        cpx<T> t3 = mul_i<DIR>(cscale(csub(b, c), s3));
        v[0] = cadd(a, t1);
        v[1] = cadd(t2, t3);
        v[2] = csub(t2, t3);
    }
};

template <int DIR, typename T>
struct Dft<4, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v)
    {
        cpx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cpx<T> s0 = cadd(a, c), d0 = csub(a, c);
        cpx<T> s1 = cadd(b, d), d1 = mul_i<DIR>(csub(b, d));
        v[0] = cadd(s0, s1);
        v[1] = cadd(d0, d1);
        v[2] = csub(s0, s1);
        v[3] = csub(d0, d1);
    }
};

template <int DIR, typename T>
struct Dft<5, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v)
    {
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        cpx<T> a = v[0];
        cpx<T> t1 = cadd(v[1], v[4]), t3 = csub(v[1], v[4]);
        cpx<T> t2 = cadd(v[2], v[3]), t4 = csub(v[2], v[3]);
        cpx<T> r1 = {a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
        cpx<T> r2 = {a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
        cpx<T> i1 = mul_i<DIR>(cpx<T>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
        cpx<T> i2 = mul_i<DIR>(cpx<T>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
        v[0] = cadd(a, cadd(t1, t2));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    }
};

// R = A * B by one Cooley-Tukey split: input n = B n1 + n2, output
// k = k1 + A k2; inner DFT_A over n1, twiddle w_R^{n2 k1}, outer DFT_B over n2.
template <int A, int B, int DIR, typename T>
struct DftSplit {
    static constexpr int R = A * B;
    template <int N2, int K1>
    __device__ __forceinline__ static void rot(cpx<T> (&y)[B][A])
    {
        y[N2][K1] = rot_const<R, N2 * K1, DIR>(y[N2][K1]);
        if constexpr (K1 + 1 < A) rot<N2, K1 + 1>(y);
        else if constexpr (N2 + 1 < B) rot<N2 + 1, 0>(y);
    }
    __device__ __forceinline__ static void run(cpx<T>* v)
    {
        cpx<T> y[B][A];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) y[n2][n1] = v[B * n1 + n2];
            Dft<A, DIR, T>::run(y[n2]);
        }
        rot<1, 1>(y);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            cpx<T> z[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) z[n2] = y[n2][k1];
            Dft<B, DIR, T>::run(z);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = z[k2];
        }
    }
};

template <int DIR, typename T>
struct Dft<8, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v) { DftSplit<2, 4, DIR, T>::run(v); }
};

template <int DIR, typename T>
struct Dft<16, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v) { DftSplit<4, 4, DIR, T>::run(v); }
};

template <int DIR, typename T>
struct Dft<6, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v) { DftSplit<2, 3, DIR, T>::run(v); }
};

template <int DIR, typename T>
struct Dft<12, DIR, T> {
    __device__ __forceinline__ static void run(cpx<T>* v) { DftSplit<4, 3, DIR, T>::run(v); }
};

// ---------------------------------------------------------------- helpers
// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Renumber them so that every XCD walks one contiguous
// range of tiles: neighbouring tiles, which share cache lines at their
// edges, then run on the same XCD at about the same time.
__device__ __forceinline__ long long xcd_tile(long long nb)
{
    const long long i = blockIdx.x;
    const long long c = nb / 8, rem = nb % 8;
    const long long x = i % 8, j = i / 8;
    return x * c + (x < rem ? x : rem) + j;
}

// ---------------------------------------------------------------- plans
template <int... Rs>
struct Radices;

template <int R0, int... Rest>
struct Radices<R0, Rest...> {
    static constexpr int first = R0;
    static constexpr int count = 1 + sizeof...(Rest);
    static constexpr int product = R0 * Radices<Rest...>::product;
    static constexpr int last = Radices<Rest...>::count == 0 ? R0 : Radices<Rest...>::last;
};
template <>
struct Radices<> {
    static constexpr int count = 0;
    static constexpr int product = 1;
    static constexpr int last = 1;
};

// LDS position of element pos of a line: one pad slot every PD elements
// breaks the stride-R bank pattern of the first exchange.
template <int PD>
__device__ __forceinline__ int lds_pos(int pos) { return pos + pos / PD; }

// LDS slot of element pos in the exchange that follows a stage of span P
// and radix R, for ES-byte LDS elements.  PD > 0: the padded layout above.
// PD == 0: a per-stage padding.  The LDS has 32 banks of 4 bytes and serves
// 8-byte accesses 16 lanes at a time (measured with rocprofv3's
// SQ_LDS_BANK_CONFLICT on gfx950: a lane stride of s slots costs 4 (s - 1)
// extra cycles per wave for s <= 16), so a conflict-free row is
// W = LDS_ROW_BYTES / ES elements.  The stage writes
// element (b - k) R + k + m P from lane b (k = b mod P); adding P slots
// after every D = max(W, P R) elements spreads the lanes that share k over
// the P-slot groups of a row, while the unit-stride reads of the next stage
// stay inside one row.  The padding is a multiple of P and constant over
// each block of D elements, so m P and the tile offsets stay immediate
// address offsets.  Stages with P >= W write at unit stride and need none.
constexpr bool pow2c(int x) { return x > 0 && (x & (x - 1)) == 0; }

constexpr int LDS_ROW_BYTES = 128;

// Period of the layout: lds_slot(x + c) = lds_slot(x) + lds_delta(c) for
// every multiple c of it.
template <int PD, int P, int R, int ES>
constexpr int lds_period()
{
    constexpr int W = LDS_ROW_BYTES / ES;
    return PD > 0 ? PD : (P >= W ? 1 : (P * R > W ? P * R : W));
}

template <int PD, int P, int R, int ES>
constexpr int lds_delta(int c)
{
    constexpr int W = LDS_ROW_BYTES / ES;
    return PD > 0 ? c + c / PD : (P >= W ? c : c + P * (c / lds_period<PD, P, R, ES>()));
}

template <int PD, int P, int R, int ES>
__device__ __forceinline__ int lds_slot(int pos)
{
    if constexpr (PD > 0) {
        return pos + pos / PD;
    } else {
        constexpr int W = LDS_ROW_BYTES / ES;
        if constexpr (P >= W) {
            return pos;
        } else {
            constexpr int D = P * R > W ? P * R : W;
            return pos + P * (pos / D);
        }
    }
}

// Synchronisation of an LDS exchange.  WS = false: the whole block.  WS =
// true: only the calling wavefront, for lines whose threads all lie in one
// wavefront; a wavefront's LDS operations are executed in program order, so
// the fences only keep the compiler from moving LDS accesses across it.
template <bool WS>
__device__ __forceinline__ void lds_sync()
{
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Stage s of a transform of length N held by G threads: compute the
// butterflies, then (unless it is the last stage) exchange through LDS into
// the register layout of the next stage.  lds points at this line's slot 0;
// element pos lives at lds[lds_slot<PD, P, R, ES>(pos) * LS].  With SP = 1 the
// exchange moves the real and then the imaginary parts through a real-valued
// buffer of the same layout (half the LDS, twice the barriers).
// DB = true: the exchanges alternate between two LDS buffers, dbo bytes
// apart, with par (kept by the caller across transforms) selecting the one
// to write next.  Every thread then finishes reading an exchange's buffer
// before it can pass the barrier of the following exchange, which writes
// the other buffer, so the barrier after the reads is not needed.
// A butterfly order for lines of 128 threads (two wavefronts) in which
// butterflies b and (128 - b) mod 128 always lie in the same wavefront:
// wavefront 0 takes 0..31, 97..127 and 64, wavefront 1 takes 32..63 and
// 65..96.  mirror_lane(b) is the lane (within its wavefront) of butterfly b.
__device__ __forceinline__ int mirror_order(int t)
{
    const int l = t & 63;
    if (t < 64) return l < 32 ? l : (l < 63 ? l + 65 : 64);
    return l < 32 ? l + 32 : l + 33;
}
__device__ __forceinline__ int mirror_lane(int b)
{
    if (b < 32) return b;
    if (b < 64) return b - 32;
    if (b == 64) return 63;
    return b < 97 ? b - 33 : b - 65;
}

template <int N, int G, int DIR, int PD, int LS, int SP, bool WS, bool DB, typename T, int P, int OFF, int... Rs>
struct Stages;

template <int N, int G, int DIR, int PD, int LS, int SP, bool WS, bool DB, typename T, int P, int OFF, int R,
          int... Rest>
struct Stages<N, G, DIR, PD, LS, SP, WS, DB, T, P, OFF, R, Rest...> {
    static constexpr int E = N / G;
    static constexpr int NB = N / (R * G);
    static_assert(NB * R * G == N, "G must divide N / R for every radix");

    // Where the layout is additive over the constant parts of the indices,
    // one slot per thread is computed and the rest are immediate offsets:
    // writes go to (t - k) R + k + (q G R + m P) with k = t mod P when P
    // divides G, and that offset never carries a row past a period boundary
    // (k + m P < P R); reads go to t + (q G + m N / R2).
    template <int ES>
    static constexpr bool fast_write()
    {
        constexpr int PER = lds_period<PD, P, R, ES>();
        if (G % P != 0 || (G * R) % PER != 0) return false;
        if (PD > 0) return P == 1 ? R % PD == 0 : P % PD == 0;
        return pow2c(P) && pow2c(R) && pow2c(PER);
    }
    template <int R2, int ES>
    static constexpr bool fast_read()
    {
        constexpr int PER = lds_period<PD, P, R, ES>();
        return G % PER == 0 && (N / R2) % PER == 0;
    }

    // (tr: the thread index that reads, i.e. the butterfly index this thread
    // takes in the next stage; t otherwise)
    template <int R2, typename L, typename Get, typename Put>
    __device__ __forceinline__ static void exchange(cpx<T> (&v)[E], int t, L* lds0, Get get, Put put, int dbo,
                                                    int& par, int tr)
    {
        constexpr int ES = sizeof(L);
        L* lds = lds0;
        if constexpr (DB) lds = reinterpret_cast<L*>(reinterpret_cast<char*>(lds0) + par * dbo);
        if constexpr (fast_write<ES>()) {
            const int k = t % P;
            L* base = lds + lds_slot<PD, P, R, ES>((t - k) * R + k) * LS;
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int m = 0; m < R; ++m) base[lds_delta<PD, P, R, ES>(q * G * R + m * P) * LS] = get(v[q * R + m]);
        } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int b = t + q * G;
                const int k = b % P;
                const int j = (b - k) * R + k;
#pragma unroll
                for (int m = 0; m < R; ++m) lds[lds_slot<PD, P, R, ES>(j + m * P) * LS] = get(v[q * R + m]);
            }
        }
        lds_sync<WS>();
        if constexpr (fast_read<R2, ES>()) {
            const L* base = lds + lds_slot<PD, P, R, ES>(tr) * LS;
#pragma unroll
            for (int q = 0; q < N / (R2 * G); ++q)
#pragma unroll
                for (int m = 0; m < R2; ++m)
                    put(v[q * R2 + m], base[lds_delta<PD, P, R, ES>(q * G + m * (N / R2)) * LS]);
        } else {
#pragma unroll
            for (int q = 0; q < N / (R2 * G); ++q)
#pragma unroll
                for (int m = 0; m < R2; ++m)
                    put(v[q * R2 + m], lds[lds_slot<PD, P, R, ES>(tr + q * G + m * (N / R2)) * LS]);
        }
        if constexpr (DB) par ^= 1;
        else lds_sync<WS>();
    }

    // The exchange before a last radix-2 stage, for a line of G = 16 or 32
    // consecutive lanes (LS = 1), when this stage has one butterfly per
    // thread (E = R) and span P = G / 2.  Thread t then holds
    // x[h N/2 + t % (G/2) + m G/2], h = t / (G/2), and butterfly q of the
    // last stage in thread t takes x[t + q G] and x[t + q G + N/2]: slot
    // 2q + h of its own lane and of lane t ^ (G/2).  So each butterfly needs
    // one value from the partner lane, which a cross-lane move brings over in
    // registers (G = 16: a DPP row rotation by 8; G = 32: ds_swizzle with
    // xor mask 16, which goes through the LDS crossbar but not LDS memory):
    // no LDS buffer and no barrier.
    template <int R2>
    static constexpr bool lane_swap()
    {
        return R2 == 2 && sizeof...(Rest) == 1 && (G == 16 || G == 32) && LS == 1 && NB == 1 && P == G / 2 &&
               DB == 0;
    }
    __device__ __forceinline__ static int swap_word(int w)
    {
        if constexpr (G == 16) return __builtin_amdgcn_mov_dpp(w, 0x128, 0xF, 0xF, false);  // row_ror:8
        else return __builtin_amdgcn_ds_swizzle(w, 0x401F);  // bit mode: and 0x1F, or 0, xor 0x10
    }
    __device__ __forceinline__ static T partner(T x)
    {
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, swap_word(__builtin_bit_cast(int, x)));
        } else {
            const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
            const unsigned lo = (unsigned)swap_word((int)(unsigned)u);
            const unsigned hi = (unsigned)swap_word((int)(unsigned)(u >> 32));
            return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
        }
    }
    __device__ __forceinline__ static void swap_exchange(cpx<T> (&v)[E], int t)
    {
        const bool h = (t & (G / 2)) != 0;
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
            // element-wise selects (a conditional store into v would be
            // turned into a dynamically indexed stack array)
            const cpx<T> a0 = v[2 * q], a1 = v[2 * q + 1];
            const T rx = partner(h ? a0.x : a1.x), ry = partner(h ? a0.y : a1.y);
            v[2 * q] = {h ? rx : a0.x, h ? ry : a0.y};
            v[2 * q + 1] = {h ? a1.x : rx, h ? a1.y : ry};
        }
    }

    template <typename L>
    __device__ __forceinline__ static void run(cpx<T> (&v)[E], int t, L* lds, const cpx<T>* __restrict__ tw, int dbo,
                                               int& par)
    {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = t + q * G;
            if constexpr (P > 1) {
                const int k = b % P;
#pragma unroll
                for (int m = 1; m < R; ++m) v[q * R + m] = twiddle<DIR>(v[q * R + m], tw[OFF + (m - 1) * P + k]);
            }
            Dft<R, DIR, T>::run(&v[q * R]);
        }
        if constexpr (sizeof...(Rest) > 0) {
            constexpr int R2 = Radices<Rest...>::first;
            if constexpr (lane_swap<R2>()) {
                swap_exchange(v, t);
            } else if constexpr (SP == 0) {
                exchange<R2>(v, t, lds, [](cpx<T> a) { return a; }, [](cpx<T>& d, cpx<T> a) { d = a; }, dbo, par, t);
            } else {
                T* l = reinterpret_cast<T*>(lds);
                exchange<R2>(v, t, l, [](cpx<T> a) { return a.x; }, [](cpx<T>& d, T a) { d.x = a; }, dbo, par, t);
                exchange<R2>(v, t, l, [](cpx<T> a) { return a.y; }, [](cpx<T>& d, T a) { d.y = a; }, dbo, par, t);
            }
            Stages<N, G, DIR, PD, LS, SP, WS, DB, T, P * R, OFF + (P > 1 ? (R - 1) * P : 0), Rest...>::run(v, t, lds, tw,
                                                                                                      dbo, par);
        }
    }

    // NV transforms of the same plan by the same thread, stage by stage:
    // each twiddle factor is read from LDS once and applied to all NV
    // (the exchanges still run one transform after the other through the
    // one buffer)
    // MIR = true: the last stage takes butterfly mirror_order(t) instead of
    // t (lines of 128 threads), so that butterflies b and G - b, whose
    // outputs hold the bins k and N - k, lie in the same wavefront.
    template <int NV, bool MIR = false, typename L>
    __device__ __forceinline__ static void run_n(cpx<T> (&v)[NV][E], int t, L* lds, const cpx<T>* __restrict__ tw,
                                                 int dbo, int& par)
    {
        static_assert(!MIR || (G == 128 && SP == 0), "mirrored last stage for lines of 128 threads");
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = t + q * G;
            if constexpr (P > 1) {
                const int k = b % P;
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    const cpx<T> w = tw[OFF + (m - 1) * P + k];
#pragma unroll
                    for (int j = 0; j < NV; ++j) v[j][q * R + m] = twiddle<DIR>(v[j][q * R + m], w);
                }
            }
#pragma unroll
            for (int j = 0; j < NV; ++j) Dft<R, DIR, T>::run(&v[j][q * R]);
        }
        if constexpr (sizeof...(Rest) > 0) {
            constexpr int R2 = Radices<Rest...>::first;
            const int tn = MIR && sizeof...(Rest) == 1 ? mirror_order(t) : t;
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                if constexpr (lane_swap<R2>() && !MIR) {
                    swap_exchange(v[j], t);
                } else if constexpr (SP == 0) {
                    exchange<R2>(v[j], t, lds, [](cpx<T> a) { return a; }, [](cpx<T>& d, cpx<T> a) { d = a; }, dbo,
                                 par, tn);
                } else {
                    T* l = reinterpret_cast<T*>(lds);
                    exchange<R2>(v[j], t, l, [](cpx<T> a) { return a.x; }, [](cpx<T>& d, T a) { d.x = a; }, dbo, par,
                                 tn);
                    exchange<R2>(v[j], t, l, [](cpx<T> a) { return a.y; }, [](cpx<T>& d, T a) { d.y = a; }, dbo, par,
                                 tn);
                }
            }
            Stages<N, G, DIR, PD, LS, SP, WS, DB, T, P * R, OFF + (P > 1 ? (R - 1) * P : 0), Rest...>::template run_n<NV,
                                                                                                              MIR>(
                v, tn, lds, tw, dbo, par);
        }
    }
};

// Per-stage twiddle tables in LDS: stage s with span P > 1 and radix R keeps
// w_{PR}^{m k} at [(m-1) P + k] (m = 1..R-1, k < P), so lanes with
// consecutive k read consecutive words and lanes with equal k broadcast.
template <int N, int P, int... Rs>
struct TwTable {
    static constexpr int len = 0;
    template <typename T>
    __device__ __forceinline__ static void fill(int, cpx<T>*, const cpx<T>* __restrict__) {}
    __device__ __forceinline__ static int src_index(int) { return 0; }
};

template <int N, int P, int R, int... Rest>
struct TwTable<N, P, R, Rest...> {
    static constexpr int here = P > 1 ? (R - 1) * P : 0;
    static constexpr int len = here + TwTable<N, P * R, Rest...>::len;
    template <typename T>
    __device__ __forceinline__ static void fill(int idx, cpx<T>* dst, const cpx<T>* __restrict__ src)
    {
        if (idx < here) {
            const int m = idx / P + 1, k = idx % P;
            dst[idx] = src[m * k * (N / (P * R))];
        } else {
            TwTable<N, P * R, Rest...>::fill(idx - here, dst + here, src);
        }
    }
    // index into the N-entry table of stage-table entry idx
    __device__ __forceinline__ static int src_index(int idx)
    {
        if (idx < here) return (idx / P + 1) * (idx % P) * (N / (P * R));
        return TwTable<N, P * R, Rest...>::src_index(idx - here);
    }
};

template <int N_, int G_, class Rad>
struct Plan;

template <int N_, int G_, int... Rs>
struct Plan<N_, G_, Radices<Rs...>> {
    static constexpr int N = N_, G = G_, E = N_ / G_;
    using Rad = Radices<Rs...>;
    static constexpr int R0 = Rad::first, RL = Rad::last;
    static_assert(Rad::product == N_, "radices must multiply to N");
    // LDS elements per line (with padding)
    static constexpr int lds_len = N_ + N_ / R0 + 1;
    // entries of the per-stage twiddle tables (at most N)
    static constexpr int tw_len = TwTable<N_, 1, Rs...>::len;

    // build the stage tables in LDS from the N-entry table exp(-2 pi i e/N)
    // (all threads of the block take part; load_tw also waits for the block)
    template <typename T>
    __device__ __forceinline__ static void fill_tw(cpx<T>* dst, const cpx<T>* __restrict__ src)
    {
        for (int i = threadIdx.x; i < tw_len; i += blockDim.x) TwTable<N_, 1, Rs...>::fill(i, dst, src);
    }
    // the same from the table of a length STRIDE * N (every STRIDE-th entry)
    template <int STRIDE, typename T>
    __device__ __forceinline__ static void fill_tw_from(cpx<T>* dst, const cpx<T>* __restrict__ src)
    {
        for (int i = threadIdx.x; i < tw_len; i += blockDim.x)
            dst[i] = src[STRIDE * TwTable<N_, 1, Rs...>::src_index(i)];
    }
    template <typename T>
    __device__ __forceinline__ static void load_tw(cpx<T>* dst, const cpx<T>* __restrict__ src)
    {
        fill_tw(dst, src);
        __syncthreads();
    }
    // the same in two halves for blocks of NT threads: fetch_tw issues the
    // global reads into registers, put_tw writes them to LDS (no barrier)
    template <int NT>
    static constexpr int tw_per_thread = (tw_len + NT - 1) / NT;
    template <int NT, typename T>
    __device__ __forceinline__ static void fetch_tw(cpx<T> (&r)[tw_per_thread<NT> > 0 ? tw_per_thread<NT> : 1],
                                                    const cpx<T>* __restrict__ src)
    {
#pragma unroll
        for (int j = 0; j < tw_per_thread<NT>; ++j) {
            // branch-free (entry 0 stands in past the end), so that r stays
            // in registers
            const int i = threadIdx.x + j * NT;
            r[j] = src[i < tw_len ? TwTable<N_, 1, Rs...>::src_index(i) : 0];
        }
    }
    template <int NT, typename T>
    __device__ __forceinline__ static void put_tw(cpx<T>* dst, const cpx<T> (&r)[tw_per_thread<NT> > 0 ? tw_per_thread<NT> : 1])
    {
#pragma unroll
        for (int j = 0; j < tw_per_thread<NT>; ++j) {
            const int i = threadIdx.x + j * NT;
            if (i < tw_len) dst[i] = r[j];
        }
    }

    // LDS elements per line with the per-stage padding (lds_slot, PD = 0)
    // for ES-byte elements
    template <int ES>
    static constexpr int lds_len_st()
    {
        constexpr int rad[] = {Rs...};
        constexpr int W = LDS_ROW_BYTES / ES;
        int P = 1, ext = N_;
        for (int s = 0; s + 1 < (int)sizeof...(Rs); ++s) {
            const int R = rad[s];
            if (P < W) {
                const int D = P * R > W ? P * R : W;
                const int e = N_ + P * ((N_ - 1) / D);
                ext = e > ext ? e : ext;
            }
            P *= R;
        }
        return ext;
    }

    // ST = true selects the per-stage padding (for LS = 1); WS = true
    // synchronises the exchanges per wavefront (the G threads of a line must
    // lie in one wavefront)
    template <int DIR, int LS, int SP = 0, bool ST = false, bool WS = false, typename T>
    __device__ __forceinline__ static void run(cpx<T> (&v)[E], int t, cpx<T>* lds, const cpx<T>* __restrict__ tw)
    {
        static_assert(!ST || (LS == 1 && SP == 0), "per-stage padding is laid out for one line at unit stride");
        static_assert(!WS || (G_ <= 64 && 64 % G_ == 0), "wavefront-synchronous exchanges need lines inside a wavefront");
        int par = 0;
        Stages<N_, G_, DIR, ST ? 0 : R0, LS, SP, WS, false, T, 1, 0, Rs...>::run(v, t, lds, tw, 0, par);
    }
    // the same for NV lines of one thread, transformed stage by stage with
    // shared twiddle reads
    // MIR = true: the last stage runs in mirror_order (its outputs for
    // thread t are X[mirror_order(t) + m N / RL])
    template <int DIR, int LS, int SP = 0, bool ST = false, bool WS = false, bool MIR = false, int NV, typename T>
    __device__ __forceinline__ static void run_n(cpx<T> (&v)[NV][E], int t, cpx<T>* lds, const cpx<T>* __restrict__ tw)
    {
        static_assert(!ST || (LS == 1 && SP == 0), "per-stage padding is laid out for one line at unit stride");
        static_assert(!WS || (G_ <= 64 && 64 % G_ == 0), "wavefront-synchronous exchanges need lines inside a wavefront");
        int par = 0;
        Stages<N_, G_, DIR, ST ? 0 : R0, LS, SP, WS, false, T, 1, 0, Rs...>::template run_n<NV, MIR>(v, t, lds, tw, 0,
                                                                                                 par);
    }
    // the same with double-buffered exchanges (the second buffer dbo bytes
    // after the first; par selects the next buffer to write and is updated)
    template <int DIR, int LS, int SP = 0, typename T>
    __device__ __forceinline__ static void run_db(cpx<T> (&v)[E], int t, cpx<T>* lds, const cpx<T>* __restrict__ tw,
                                                  int dbo, int& par)
    {
        Stages<N_, G_, DIR, R0, LS, SP, false, true, T, 1, 0, Rs...>::run(v, t, lds, tw, dbo, par);
    }
    // exchanges per transform (each split exchange counts twice)
    static constexpr int exchanges(int sp) { return (int)(sizeof...(Rs) - 1) * (sp ? 2 : 1); }
    // position of register element i = q * R + m at stage-0 input / final output
    __device__ __forceinline__ static constexpr int in_pos(int t, int i) { return t + (i / R0) * G + (i % R0) * (N / R0); }
    __device__ __forceinline__ static constexpr int out_pos(int t, int i) { return t + (i / RL) * G + (i % RL) * (N / RL); }
    // Both sets are {t + k G : k < E}: in_pos has k = i / R0 + (i % R0) (E / R0)
    // and out_pos k = i / RL + (i % RL) (E / RL).  out_slot_of_in(i) is the
    // output slot whose position is the input position of slot i, so an
    // output can be fed to a second transform of the same plan without
    // leaving the thread.
    static constexpr int out_slot_of_in(int i)
    {
        const int k = i / R0 + (i % R0) * (E / R0);
        return (k % (E / RL)) * RL + k / (E / RL);
    }
    static constexpr bool slot_map_ok()
    {
        for (int i = 0; i < E; ++i) {
            const int o = out_slot_of_in(i);
            if (o < 0 || o >= E || i / R0 + (i % R0) * (E / R0) != o / RL + (o % RL) * (E / RL)) return false;
        }
        return true;
    }
};

}  // namespace ns
