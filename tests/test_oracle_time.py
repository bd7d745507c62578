"""Pins of the oracle's SSP-RK3 stepper and its discrete adjoint."""
import numpy as np
import pytest

from paper_2401_09843_amd import inputs


def fdot(orc, a, b, n):
    """<a, b> = Re sum_k conj(a_k) b_k over the full spectrum."""
    return float(np.real(np.vdot(orc.full_from_r2c(a, n), orc.full_from_r2c(b, n))))


def test_rk3_linear_amplification_polynomial(orc):
    # a single damped mode with F = lambda u: one step multiplies by
    # 1 + z + z^2/2 + z^3/6; each of the three stage weights changes it
    n = 16
    x, y, z = inputs.grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = np.cos(4 * y)
    uh = orc.forward(u)
    eps, dt = 0.05, 0.02
    lam = -eps * 4.0 ** 3
    zz = dt * lam
    out = orc.ssprk3(uh, n, dt, 1, orc.Params(eps=eps, m_cut=1.0))
    assert np.max(np.abs(out - (1 + zz + zz ** 2 / 2 + zz ** 3 / 6) * uh)) <= 1e-16


def test_rk3_third_order_on_taylor_green(orc):
    n, T = 16, 0.4
    uh = orc.initial_state(inputs.taylor_green(n))
    ref = orc.ssprk3(uh, n, T / 64, 64, orc.Params(eps=0.0))
    errs = []
    for steps in (4, 8, 16):
        errs.append(np.linalg.norm(orc.ssprk3(uh, n, T / steps, steps, orc.Params(eps=0.0)) - ref))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 2.8) and np.all(orders < 3.3), orders


def test_inviscid_energy_drift_is_small_and_nonincreasing(orc):
    n = 16
    u, _, _ = inputs.shear_layer(n, seed=0, rho=0.2)
    uh = orc.initial_state(u)
    dt = inputs.cfl_dt(u)

    def energy(h):
        return 0.5 * fdot(orc, h, h, n)

    e0 = energy(uh)
    e = [e0]
    h = uh
    for _ in range(5):
        h = orc.ssprk3(h, n, dt, 1, orc.Params(eps=0.0))
        e.append(energy(h))
    e = np.array(e)
    assert np.all(np.diff(e) <= 0.0)
    assert np.all(np.abs(e - e0) <= 1e-4 * e0)
    assert orc.div_rel(h, n) <= 1e-13


def test_vjp_dot_product_identity(orc):
    # F is quadratic, so the central difference is exact up to rounding
    n = 12
    prm = orc.Params(eps=3e-3, m_cut=2.0)
    uh = inputs.half_spectrum(inputs.random_field(n, seed=41))
    v = inputs.half_spectrum(inputs.random_field(n, seed=42))
    lam = inputs.half_spectrum(inputs.random_field(n, seed=43))
    h = 1e-2
    jv = (orc.rhs(uh + h * v, n, prm) - orc.rhs(uh - h * v, n, prm)) / (2 * h)
    jtl = orc.rhs_vjp(uh, lam, n, prm)
    lhs, rhs = fdot(orc, lam, jv, n), fdot(orc, jtl, v, n)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_vjp_full_jacobian_small(orc):
    # N = 6 (K = 1): every column of the Jacobian by central differences
    n = 6
    prm = orc.Params(eps=1e-2, m_cut=0.5)
    uh = orc.initial_state(inputs.random_field(n, seed=44))
    lam = inputs.half_spectrum(inputs.random_field(n, seed=45))
    g = orc.rhs_vjp(uh, lam, n, prm)
    # real-space directions are the independent coordinates; compare
    # <lam, J e> with <J^T lam, e> for many unit fields e
    rng = np.random.default_rng(0)
    for _ in range(12):
        e = np.zeros((3, n, n, n))
        e[rng.integers(3), rng.integers(n), rng.integers(n), rng.integers(n)] = 1.0
        eh = inputs.half_spectrum(e)
        jv = (orc.rhs(uh + 0.5 * eh, n, prm) - orc.rhs(uh - 0.5 * eh, n, prm))
        assert abs(fdot(orc, lam, jv, n) - fdot(orc, g, eh, n)) <= 1e-13


def test_adjoint_step_matches_finite_differences(orc):
    n = 12
    prm = orc.Params(eps=3e-3, m_cut=2.0)
    u = inputs.random_field(n, seed=51)
    uh = orc.initial_state(u)
    dt = 0.5 * inputs.cfl_dt(u)
    lam = inputs.half_spectrum(inputs.random_field(n, seed=52))
    g = orc.adjoint_step(uh, lam, n, dt, prm)
    for seed in (53, 54):
        v = inputs.half_spectrum(inputs.random_field(n, seed=seed))
        h = 1e-4
        d = (orc.ssprk3(uh + h * v, n, dt, 1, prm) - orc.ssprk3(uh - h * v, n, dt, 1, prm)) / (2 * h)
        lhs, rhs = fdot(orc, lam, d, n), fdot(orc, g, v, n)
        assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_rollout_gradient_matches_finite_differences(orc):
    # the reference gradient through T P F, three SSP-RK3 steps and a shell
    # energy objective, against central differences along physical directions
    n, steps = 12, 3
    prm = orc.Params(eps=2e-3, m_cut=2.0)
    u0 = inputs.random_field(n, seed=61)
    dt = 0.5 * inputs.cfl_dt(u0)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, np.arange(n // 2 + 1), indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    w = ((kk >= 2) & (kk < 4)).astype(float)
    J0, g = orc.rollout_gradient(u0, dt, steps, w, prm)

    def J(u):
        uh = orc.ssprk3(orc.initial_state(u, prm), n, dt, steps, prm)
        full = orc.full_from_r2c(uh, n)
        wf = np.real(orc.full_from_r2c(w[None].astype(complex), n))[0]
        return 0.5 * np.sum(wf[None] * np.abs(full) ** 2)

    assert abs(J(u0) - J0) <= 1e-14 * abs(J0)
    for seed in (62, 63):
        v = inputs.random_field(n, seed=seed)
        h = 1e-4
        fd = (J(u0 + h * v) - J(u0 - h * v)) / (2 * h)
        assert abs(fd - np.sum(g * v)) <= 1e-8 * abs(fd)
