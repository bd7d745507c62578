"""Pins of the oracle's transforms against the DFT's definition and against
an independent library FFT (numpy's pocketfft, which the oracle never calls)."""
import numpy as np
import pytest

from paper_2401_09843_amd import inputs


def dft_matrix(n, sign):
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


@pytest.mark.parametrize("n", list(range(1, 17)) + [18, 20, 24, 25, 27, 30, 32, 45, 48, 60, 64, 80, 96, 120])
@pytest.mark.parametrize("sign", [-1, 1])
def test_dft1_matches_definition(orc, n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = dft_matrix(n, sign) @ x
    got = orc.dft1(x, sign)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8])
def test_fft3_matches_brute_force(orc, n):
    rng = np.random.default_rng(100 + n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    for sign in (-1, 1):
        ref = orc.dft3_brute(a, sign)
        assert np.max(np.abs(orc.fft3(a, sign) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_brute_dft3_is_the_definition(orc):
    # the O(N^6) routine against a Kronecker product of 1-D DFT matrices
    n = 4
    rng = np.random.default_rng(7)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    W = dft_matrix(n, -1)
    ref = np.einsum("ai,bj,ck,ijk->abc", W, W, W, a)
    assert np.allclose(orc.dft3_brute(a, -1), ref, atol=1e-12)


@pytest.mark.parametrize("n", [8, 12, 16, 20, 30, 32])
def test_fft3_matches_library_fft(orc, n):
    rng = np.random.default_rng(200 + n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    ref = np.fft.fftn(a)
    assert np.max(np.abs(orc.fft3(a, -1) - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [8, 12, 16, 24])
def test_forward_is_normalised_half_spectrum(orc, n):
    u = inputs.random_field(n, seed=n)
    ref = np.fft.rfftn(u, axes=(-3, -2, -1), norm="forward")
    got = orc.forward(u)
    assert np.max(np.abs(got - ref)) <= 1e-14 * n ** 3 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [8, 10, 16])
def test_inverse_forward_roundtrip(orc, n):
    u = inputs.random_field(n, seed=3 * n)
    back = orc.inverse(orc.forward(u), n)
    assert np.max(np.abs(back - u)) <= 1e-13


def test_single_mode_closed_form(orc):
    # cos(3x - 2y + z) has coefficients 1/2 at +-(3,-2,1) and nothing else
    n = 16
    x, y, z = inputs.grid(n)
    u = np.zeros((3, n, n, n))
    u[1] = np.cos(3 * x - 2 * y + z)
    h = orc.forward(u)
    expect = np.zeros_like(h)
    expect[1, 1, (-2) % n, 3] = 0.5
    assert np.max(np.abs(h - expect)) <= 1e-15


def test_layout_roundtrip(orc):
    n = 12
    u = inputs.random_field(n, seed=5)
    h = np.fft.rfftn(u, axes=(-3, -2, -1), norm="forward")
    full = orc.full_from_r2c(h, n)
    assert np.allclose(full, np.fft.fftn(u, axes=(-3, -2, -1), norm="forward"), atol=1e-15)
