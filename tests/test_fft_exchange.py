"""Host check of the register exchange the FFT engine does by cross-lane
moves (a DPP row rotation for 16-thread lines, ds_swizzle for 32): when the
second-to-last stage has one butterfly per thread (E = R) and span P = G/2
and the last stage is radix 2, every value a thread needs for its last-stage
butterflies is either in its own registers or in lane t ^ (G/2) (slot
2q + h, h = t / (G/2)).  The index maps are the Stockham ones of the engine: a stage of
span P and radix R writes output m of butterfly b to (b - k) R + k + m P,
k = b mod P, and the next stage of radix R2 reads t + q G + m N / R2."""
import itertools

import pytest


def holdings(N, G, radices):
    """Position -> (thread, slot) after all stages but the last."""
    E = N // G
    assert all(E % R == 0 for R in radices), "each radix must divide the elements per thread"
    P = 1
    pos = {}
    for s, R in enumerate(radices[:-1]):
        NB = N // (R * G)
        pos = {}
        for t in range(G):
            for q in range(NB):
                b = t + q * G
                k = b % P
                for m in range(R):
                    pos[(b - k) * R + k + m * P] = (t, q * R + m)
        P *= R
    assert sorted(pos) == list(range(N))
    return pos, P, E


@pytest.mark.parametrize("N, G, radices", [(128, 16, (8, 8, 2)), (256, 16, (8, 16, 2)), (128, 32, (4, 4, 4, 2))])
def test_last_radix2_exchange_is_a_lane_swap(N, G, radices):
    pos, P, E = holdings(N, G, radices)
    R = radices[-2]
    if not (N // (R * G) == 1 and P // R == G // 2):
        pytest.skip("the engine takes the LDS exchange for this plan")
    for t in range(G):
        h = t // (G // 2)
        for q in range(E // 2):
            b = t + q * G
            for m, p in enumerate((b, b + N // 2)):
                src_t, src_slot = pos[p]
                assert src_slot == 2 * q + h
                own = (m == 0 and h == 0) or (m == 1 and h == 1)
                assert src_t == (t if own else t ^ (G // 2)), (t, q, m)


@pytest.mark.parametrize("N, radices", [(256, (16, 8, 2)), (256, (8, 4, 4, 2))])
def test_wider_spans_keep_the_values_in_their_lane(N, radices):
    """With the second-to-last span P >= G (several butterflies per thread)
    every value of a thread's last-stage butterflies is already its own: the
    swap is needed only for P = G / 2."""
    G = 16
    pos, P, E = holdings(N, G, radices)
    assert P // radices[-2] >= G
    for t, q in itertools.product(range(G), range(E // 2)):
        b = t + q * G
        for p in (b, b + N // 2):
            assert pos[p][0] == t


# ------------------------------------------------------------ mirrored order
# The x pass's grouped forward transforms can run their last stage with
# butterfly mirror_order(t) on thread t (lines of 128 threads, last radix
# E = 8), so that a thread's bins k = b + 128 m and the bins N - k it needs
# for the real-to-complex unpack lie in one wavefront.  These restate the
# engine's two index functions and check the properties the unpack relies on.
def mirror_order(t):
    l = t & 63
    if t < 64:
        return l if l < 32 else (l + 65 if l < 63 else 64)
    return l + 32 if l < 32 else l + 33


def mirror_lane(b):
    if b < 32:
        return b
    if b < 64:
        return b - 32
    if b == 64:
        return 63
    return b - 33 if b < 97 else b - 65


def test_mirror_order_is_a_permutation_with_mirror_pairs_in_one_wavefront():
    G = 128
    order = [mirror_order(t) for t in range(G)]
    assert sorted(order) == list(range(G))
    for t in range(G):
        b = order[t]
        assert mirror_lane(b) == t % 64
        partner = (G - b) % G
        tp = order.index(partner)
        assert tp // 64 == t // 64, (t, b, partner)  # same wavefront
        assert mirror_lane(partner) == tp % 64


@pytest.mark.parametrize("N, G, radices", [(1024, 128, (8, 4, 4, 8)), (512, 64, (8, 8, 8)), (128, 16, (8, 2, 8))])
def test_register_unpack_finds_each_mirror_bin_in_its_wavefront(N, G, radices):
    """The last stage runs butterfly b = mirror_order(t) (lines of 128
    threads) or b = t (lines inside one wavefront): thread t then holds
    X[b + G m] in slot m, and bin N - (b + G m) sits in slot E - 1 - m of
    the lane the kernel computes for butterfly (G - b) mod G (b != 0), or in
    slot (E - m) mod E of the thread itself (b = 0).  Several lines share a
    wavefront when G < 64; the block's thread index is u G + t for line u."""
    E = N // G
    assert radices[-1] == E and E * G == N
    K = (N - 1) // 3
    assert K < 3 * G
    order = (lambda t: mirror_order(t)) if G == 128 else (lambda t: t)
    lines = max(1, 64 // G) * 2
    held = {}
    for u in range(lines):
        for t in range(G):
            b = order(t)
            for m in range(E):
                held[(u, b + m * G)] = (u * G + t, m)
    for u in range(lines):
        assert sorted(k for (uu, k) in held if uu == u) == list(range(N))
        for t in range(G):
            tid = u * G + t
            b = order(t)
            pg = (G - b) % G
            lane = mirror_lane(pg) if G == 128 else (tid & 63) - t + pg
            for m in range(3):
                k = b + m * G
                if k > K:
                    continue
                src_tid, src_slot = held[(u, (N - k) % N)]
                if b == 0:
                    assert (src_tid, src_slot) == (tid, (E - m) % E)
                else:
                    assert src_tid // 64 == tid // 64, (u, t, m)  # same wavefront
                    assert src_tid % 64 == lane
                    assert src_slot == E - 1 - m
