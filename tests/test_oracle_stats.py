"""Pins of the oracle's in-situ statistics: the enstrophy spectrum (Sec.
2.4's writers) against closed forms, and the pointwise mean and variance of
the empirical measure (Algorithm 1, step 3) against ensembles whose moments
are known exactly."""
import numpy as np
import pytest

from paper_2401_09843_amd import inputs


@pytest.mark.parametrize("k0", [1, 2, 3])
def test_enstrophy_of_abc_flow_is_k0_squared_energy(orc, k0):
    """curl u = k0 u for an ABC flow, so Z(kappa) = k0^2 E(kappa) shell by shell."""
    n = 16
    uh = orc.forward(inputs.abc_flow(n, k0=k0, A=1.0, B=0.7, C=0.4))
    E = orc.energy_spectrum(uh, n, 12)
    Z = orc.enstrophy_spectrum(uh, n, 12)
    assert np.max(np.abs(Z - k0 ** 2 * E)) <= 1e-14 * Z.sum()
    assert Z.sum() > 0


def test_enstrophy_of_taylor_green(orc):
    """omega = (-cos x sin y sin z, -sin x cos y sin z, 2 sin x sin y cos z):
    mean |omega|^2 = 3/4, all in the shell round(sqrt 3) = 2."""
    n = 16
    Z = orc.enstrophy_spectrum(orc.forward(inputs.taylor_green(n)), n, 8)
    assert abs(Z[2] - 3.0 / 8.0) <= 1e-15
    assert np.sum(np.abs(np.delete(Z, 2))) <= 1e-15


def test_moments_of_closed_form_ensembles(orc):
    n = 8
    u = inputs.random_field(n, seed=1)
    c = inputs.random_field(n, seed=2)
    # {u, -u}: mean 0, variance u^2
    mean, var = orc.moments([orc.forward(u), orc.forward(-u)], n)
    assert np.max(np.abs(mean)) <= 1e-15 and np.max(np.abs(var - u * u)) <= 1e-14
    # u + b c for b = 0..B-1: mean u + c (B-1)/2, variance c^2 (B^2-1)/12
    B = 5
    mean, var = orc.moments([orc.forward(u + b * c) for b in range(B)], n)
    assert np.max(np.abs(mean - (u + c * (B - 1) / 2))) <= 1e-13
    assert np.max(np.abs(var - c * c * (B * B - 1) / 12)) <= 1e-13


def test_wasserstein_closed_forms(orc):
    rng = np.random.default_rng(0)
    a = rng.standard_normal((7, 50))
    assert np.max(np.abs(orc.wasserstein1_pointwise(a, a))) == 0.0
    # a shift by c moves every quantile by c
    assert np.max(np.abs(orc.wasserstein1_pointwise(a, a + 0.3) - 0.3)) <= 1e-14
    # equal counts: the mean distance between order statistics
    b = rng.standard_normal((7, 50))
    ref = np.mean(np.abs(np.sort(a, axis=0) - np.sort(b, axis=0)), axis=0)
    assert np.max(np.abs(orc.wasserstein1_pointwise(a, b) - ref)) <= 1e-14
    # unequal counts: point masses {0} and {0, 1}: half the mass moves by 1
    assert abs(orc.wasserstein1_pointwise(np.zeros((1, 1)), np.array([[0.0], [1.0]]))[0] - 0.5) <= 1e-15


def test_wasserstein_matches_scipy(orc):
    """The textbook routine for unequal ensembles (scipy.stats)."""
    from scipy.stats import wasserstein_distance
    rng = np.random.default_rng(1)
    a = rng.standard_normal((5, 40))
    b = 0.5 + 2.0 * rng.standard_normal((9, 40))
    got = orc.wasserstein1_pointwise(a, b)
    ref = np.array([wasserstein_distance(a[:, i], b[:, i]) for i in range(40)])
    assert np.max(np.abs(got - ref)) <= 1e-14


def test_structure_functions_of_a_sine(orc):
    """u = (sin kX, 0, 0): the increment along x is 2 cos(kX + a) sin a with
    a = pi k l / n, so S_2 = (2/3) sin^2 a and S_4 = 2 sin^4 a (grid means of
    cos^2 and cos^4 are 1/2 and 3/8 when n does not divide 4k)."""
    n, k = 16, 3
    X, Y, Z = inputs.grid(n)
    u = np.stack([np.sin(k * X), 0 * X, 0 * X])
    uh = orc.forward(u)
    l = np.arange(1, 9)
    a = np.pi * k * l / n
    assert np.max(np.abs(orc.structure_functions(uh, n, 8, 2.0) - 2.0 / 3.0 * np.sin(a) ** 2)) <= 1e-14
    assert np.max(np.abs(orc.structure_functions(uh, n, 8, 4.0) - 2.0 * np.sin(a) ** 4)) <= 1e-14


def test_structure_functions_symmetry(orc):
    """A shift by l and by n - l average the same increments."""
    n = 12
    uh = orc.forward(inputs.random_field(n, seed=4))
    S = orc.structure_functions(uh, n, n - 1, 1.5)
    assert np.max(np.abs(S - S[::-1])) <= 1e-14 * S.max()
