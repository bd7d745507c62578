"""Pins of the oracle's padded form of Algorithm 2 (n modes per axis,
products on a grid of npad >= 3n/2 points): the Galerkin triad sum over the
retained modes (what an alias-free product reaches exactly), independence of
the padded size (Sec. 3.1: any size above 3n/2 serves), agreement with the
2/3-rule oracle run on the padded grid, and closed-form flows."""
import numpy as np
import pytest

from paper_2401_09843_amd import inputs
from test_oracle_rhs import triad_rhs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [8, 12, 16])
def test_padded_rhs_equals_triad_sum(orc, n):
    prm = orc.Params(eps=2e-3, m_cut=1.5)
    uh = inputs.half_spectrum(inputs.random_field(n, seed=40 + n))
    got = orc.rhs_padded(uh, n, 3 * n // 2, prm)
    ref = triad_rhs(uh, n, orc.padded_cutoff(n), 2e-3, 1.5, 1.5)
    assert rel(got, ref) <= 1e-13


def test_padded_size_does_not_matter_above_three_halves(orc):
    n = 16
    prm = orc.Params(eps=1e-3, m_cut=2.0)
    uh = inputs.half_spectrum(inputs.random_field(n, seed=7))
    ref = orc.rhs_padded(uh, n, 24, prm)
    for npad in (25, 27, 30, 32):
        assert rel(orc.rhs_padded(uh, n, npad, prm), ref) <= 1e-13, npad
    with pytest.raises(ValueError):
        orc.rhs_padded(uh, n, 23, prm)


@pytest.mark.parametrize("n", [8, 16, 20])
def test_padded_equals_two_thirds_oracle_on_the_padded_grid(orc, n):
    """The 2/3-rule oracle (C, recursive FFT) on the 3n/2 grid with cutoff
    n/2 - 1 is the same method: the two implementations share nothing but
    the layout helpers."""
    npad = 3 * n // 2
    K = orc.padded_cutoff(n)
    uh = inputs.half_spectrum(inputs.random_field(n, seed=90 + n))
    got = orc.rhs_padded(uh, n, npad, orc.Params(eps=1e-3, m_cut=2.0, q_kind=1, theta=1.3))
    ref = orc.crop_padded(orc.rhs(orc.embed_padded(uh, n, npad), npad,
                                  orc.Params(eps=1e-3, m_cut=2.0, q_kind=1, theta=1.3, kcut=K)), n, npad)
    assert rel(got, ref) <= 1e-13
    # the Nyquist planes of the n-mode layout stay zero
    assert np.all(got[:, n // 2] == 0) and np.all(got[:, :, n // 2] == 0) and np.all(got[..., n // 2] == 0)


def test_padded_taylor_green_closed_form(orc):
    n = 16
    u0 = inputs.taylor_green(n)
    uh = orc.forward(u0)
    F = orc.rhs_padded(uh, n, 24, orc.Params(eps=1e-3))
    x, y, z = inputs.grid(n)
    expect = np.stack([-np.sin(2 * x) * np.cos(2 * z) / 8, -np.sin(2 * y) * np.cos(2 * z) / 8,
                       (np.cos(2 * x) + np.cos(2 * y)) * np.sin(2 * z) / 8])
    assert np.max(np.abs(orc.inverse(F, n) - expect)) <= 1e-14


def test_padded_beltrami_mode_only_decays(orc):
    """A single helical mode: the nonlinear term is a gradient, removed by
    the projection, so F = -eps |k|^{2s} u-hat exactly."""
    n, k = 16, (3, 3, 3)
    eps = 1e-3
    uh = orc.forward(inputs.helical_mode(n, k=k))
    F = orc.rhs_padded(uh, n, 24, orc.Params(eps=eps, m_cut=1.0))
    rate = eps * (3 * 9.0) ** 1.5
    assert rel(F, -rate * uh) <= 1e-13
