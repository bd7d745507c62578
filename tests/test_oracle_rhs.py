"""Pins of the oracle's right-hand side, projection and diagnostics against
what the paper and the mathematics fix: the Galerkin triad sum (the plain
definition that a 2/3-dealiased pseudo-spectral product reaches exactly),
closed-form flows, invariants and symmetries."""
import numpy as np
import pytest

from paper_2401_09843_amd import inputs


def wn(n):
    return np.fft.fftfreq(n, 1.0 / n).astype(np.int64)


def triad_rhs(uh, n, K, eps, s, m_cut):
    """Galerkin right-hand side summed over triads p + q = k with p, q, k in
    the cube |.|_inf <= K, then the Leray projection and the step-multiplier
    hyperviscosity.  Brute force, numpy, independent of the oracle."""
    full = np.fft.fftn(np.fft.irfftn(uh, s=(n, n, n), axes=(-3, -2, -1), norm="forward"),
                       axes=(-3, -2, -1), norm="forward")
    ks = np.arange(-K, K + 1)
    P = np.array([(a, b, c) for c in ks for b in ks for a in ks])  # (kx, ky, kz)
    idx = (P[:, 2] % n, P[:, 1] % n, P[:, 0] % n)
    U = np.stack([full[i][idx] for i in range(3)])  # [3][|T|]
    kk = P[:, None, :] + P[None, :, :]
    ok = np.all(np.abs(kk) <= K, axis=-1)
    pos = {tuple(p): t for t, p in enumerate(P)}
    tgt = np.array([pos.get(tuple(v), -1) for v in kk[ok]])
    b = np.zeros((3, len(P)), dtype=np.complex128)
    for i in range(3):
        for j in range(3):
            prod = (U[i][:, None] * U[j][None, :])[ok]
            conv = np.zeros(len(P), dtype=np.complex128)
            np.add.at(conv, tgt, prod)
            b[i] += -1j * P[:, j] * conv
    k2 = np.sum(P * P, axis=1).astype(np.float64)
    kb = np.sum(P.T * b, axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        c = b - np.where(k2 > 0, P.T * kb / np.where(k2 > 0, k2, 1.0), 0.0)
    kabs = np.sqrt(k2)
    rate = eps * k2 ** s * (kabs > m_cut)
    c = c - rate * U
    out = np.zeros((3, n, n, n), dtype=np.complex128)
    for i in range(3):
        out[i][idx] = c[i]
    return out[..., : n // 2 + 1]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [8, 12, 16, 18, 20])
def test_rhs_equals_triad_sum(orc, n):
    prm = orc.Params(eps=2e-3, m_cut=1.5)
    r = prm.resolved(n)
    uh = inputs.half_spectrum(inputs.random_field(n, seed=n))
    got = orc.rhs(uh, n, prm)
    ref = triad_rhs(uh, n, orc.kcut(n), r.eps, r.s, r.m_cut)
    assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("n", [12, 18])
def test_cutoff_off_by_one_aliases(orc, n):
    # with K = N/3 (3K >= N) the pseudo-spectral product aliases into T and
    # must visibly differ from the triad sum with the same K
    K = n // 3
    prm = orc.Params(eps=0.0, kcut=K)
    uh = inputs.half_spectrum(inputs.random_field(n, seed=11))
    got = orc.rhs(uh, n, prm)
    ref = triad_rhs(uh, n, K, 0.0, 1.5, 1e9)
    assert rel(got, ref) > 1e-3


def test_taylor_green_closed_form(orc):
    n = 32
    uh = orc.initial_state(inputs.taylor_green(n))
    F = orc.rhs(uh, n, orc.Params(eps=1e-3))
    x, y, z = inputs.grid(n)
    expect = np.stack([-np.sin(2 * x) * np.cos(2 * z) / 8, -np.sin(2 * y) * np.cos(2 * z) / 8,
                       (np.cos(2 * x) + np.cos(2 * y)) * np.sin(2 * z) / 8])
    assert np.max(np.abs(orc.inverse(F, n) - expect)) <= 1e-14


@pytest.mark.parametrize("k0", [1, 3])
def test_abc_flow_nonlinear_term_is_gradient(orc, k0):
    n = 24
    uh = orc.initial_state(inputs.abc_flow(n, k0=k0, A=1.0, B=0.7, C=0.4))
    eps, s = 1e-2, 1.5
    # default m_N = N/3 = 8 > k0: no damping, the flow is steady
    F = orc.rhs(uh, n, orc.Params(eps=eps))
    assert np.max(np.abs(F)) <= 1e-15
    # m_N below k0: pure hyperviscous decay at rate eps k0^(2s)
    F = orc.rhs(uh, n, orc.Params(eps=eps, m_cut=0.5))
    assert np.max(np.abs(F + eps * k0 ** (2 * s) * uh)) <= 1e-15


def test_helical_mode_decays_by_rk3_factor(orc):
    n, dt, nsteps = 32, 0.01, 10
    eps, s = 1e-3, 1.5
    uh = orc.initial_state(inputs.helical_mode(n, k=(7, 7, 7)))
    k2 = 3 * 49.0
    assert np.sqrt(k2) > n / 3
    zeta = -dt * eps * k2 ** s
    R = 1 + zeta + zeta ** 2 / 2 + zeta ** 3 / 6
    out = orc.ssprk3(uh, n, dt, nsteps, orc.Params(eps=eps))
    assert np.max(np.abs(out - R ** nsteps * uh)) <= 1e-13 * np.max(np.abs(uh))


def test_shear_base_is_pure_hyperviscosity(orc):
    n = 24
    x, y, z = inputs.grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = inputs.shear_profile(y, 0.2)
    uh = orc.forward(u)
    K = orc.kcut(n)
    prm = orc.Params(eps=1e-2, m_cut=2.5)
    F = orc.rhs(uh, n, prm)
    ky = wn(n)
    keep = np.abs(ky) <= K
    rate = 1e-2 * np.abs(ky.astype(float)) ** 3 * (np.abs(ky) > 2.5)
    expect = np.zeros_like(uh)
    expect[0, 0, :, 0] = np.where(keep, -rate * uh[0, 0, :, 0], 0)
    assert np.max(np.abs(F - expect)) <= 1e-16


def test_two_dimensional_flow_stays_two_dimensional(orc):
    # 2-D data held constant along z stays 2-D; 2-D Taylor-Green is steady
    n = 16
    uh = orc.initial_state(inputs.taylor_green_2d(n))
    F = orc.rhs(uh, n)
    assert np.max(np.abs(F)) <= 1e-15
    u, _, _ = inputs.shear_layer(n, seed=1, rho=0.2)
    u[:, :, :, :] = u[:, :1, :, :]
    u[2] = 0.0
    uh = orc.initial_state(u)
    out = orc.ssprk3(uh, n, 0.01, 3)
    assert np.max(np.abs(out[:, 1:, :, :])) <= 1e-16
    assert np.max(np.abs(out[2])) <= 1e-16


@pytest.mark.parametrize("n", [12, 16])
def test_rhs_is_divergence_free_and_truncated(orc, n):
    # the nonlinear part is projected; the hyperviscous part keeps the
    # input's divergence, so a divergence-free input gives a free output
    uh = inputs.half_spectrum(inputs.random_field(n, seed=21))
    F = orc.rhs(uh, n, orc.Params(eps=0.0))
    assert orc.div_rel(F, n) <= 1e-14
    F = orc.rhs(orc.project(uh, n), n, orc.Params(eps=1e-2, m_cut=1.0))
    assert orc.div_rel(F, n) <= 1e-14
    K = orc.kcut(n)
    k = wn(n)
    outside = (np.abs(k)[:, None, None] > K) | (np.abs(k)[None, :, None] > K) | (np.arange(n // 2 + 1)[None, None, :] > K)
    assert np.max(np.abs(F[:, outside])) == 0.0


def test_projection_is_idempotent_and_orthogonal(orc):
    n = 12
    uh = inputs.half_spectrum(inputs.random_field(n, seed=4))
    p1 = orc.project(uh, n)
    assert orc.div_rel(p1, n) <= 1e-15
    assert np.max(np.abs(orc.project(p1, n) - p1)) <= 1e-15
    # a pure gradient field projects to zero (except the mean)
    x, y, z = inputs.grid(n)
    phi = np.sin(2 * x + y) + np.cos(z - 3 * y)
    g = np.stack([2 * np.cos(2 * x + y), np.cos(2 * x + y) + 3 * np.sin(z - 3 * y), -np.sin(z - 3 * y)])
    assert np.max(np.abs(orc.project(orc.forward(g), n))) <= 1e-15


@pytest.mark.parametrize("n", [12, 16])
def test_inviscid_energy_identity(orc, n):
    uh = orc.initial_state(inputs.random_field(n, seed=31))
    F = orc.rhs(uh, n, orc.Params(eps=0.0))
    full_u = orc.full_from_r2c(uh, n)
    full_f = orc.full_from_r2c(F, n)
    dot = np.real(np.vdot(full_u, full_f))
    assert abs(dot) <= 1e-14 * np.linalg.norm(full_u) * np.linalg.norm(full_f)


def test_translation_equivariance(orc):
    n = 12
    u = inputs.random_field(n, seed=8)
    F = orc.inverse(orc.rhs(inputs.half_spectrum(u), n, orc.Params(eps=5e-3, m_cut=2.0)), n)
    us = np.roll(u, shift=(1, 2, 3), axis=(1, 2, 3))
    Fs = orc.inverse(orc.rhs(inputs.half_spectrum(us), n, orc.Params(eps=5e-3, m_cut=2.0)), n)
    assert np.max(np.abs(Fs - np.roll(F, shift=(1, 2, 3), axis=(1, 2, 3)))) <= 1e-12


def test_axis_permutation_equivariance(orc):
    # swap x <-> z in coordinates and components
    n = 12
    u = inputs.random_field(n, seed=9)
    F = orc.inverse(orc.rhs(inputs.half_spectrum(u), n), n)
    up = np.ascontiguousarray(np.transpose(u, (0, 3, 2, 1))[::-1])
    Fp = orc.inverse(orc.rhs(inputs.half_spectrum(up), n), n)
    assert np.max(np.abs(Fp - np.transpose(F, (0, 3, 2, 1))[::-1])) <= 1e-12


def test_q_kind_lower_bound_multiplier(orc):
    # Q = 1 - (m/|k|)^((2s-1)/theta) above m: single mode at (5,0,0), s=1.5
    n, m, theta, eps = 16, 3.0, 0.5, 1e-2
    x, y, z = inputs.grid(n)
    u = np.zeros((3, n, n, n))
    u[1] = np.cos(5 * x)
    uh = orc.forward(u)
    F = orc.rhs(uh, n, orc.Params(eps=eps, m_cut=m, q_kind=1, theta=theta))
    q = 1 - (m / 5.0) ** ((2 * 1.5 - 1) / theta)
    assert np.max(np.abs(F + eps * 5.0 ** 3 * q * uh)) <= 1e-15


def test_energy_spectrum_parseval_and_shells(orc):
    n = 16
    u = inputs.random_field(n, seed=12)
    uh = inputs.half_spectrum(u)
    E = orc.energy_spectrum(uh, n, 40)
    assert abs(E.sum() - 0.5 * np.mean(np.sum(u * u, axis=0))) <= 1e-13
    x, y, z = inputs.grid(n)
    v = np.zeros((3, n, n, n))
    v[2] = 2.0 * np.cos(3 * x + 4 * y)  # |k| = 5, energy 1/2 * 2 * |1|^2 = 1
    E = orc.energy_spectrum(inputs.half_spectrum(v), n, 10)
    expect = np.zeros(10)
    expect[5] = 1.0
    assert np.max(np.abs(E - expect)) <= 1e-14


@pytest.mark.parametrize("n", [12, 16, 24])
def test_sparse_triad_rhs_matches_pseudo_spectral(orc, n):
    # the sparse Galerkin evaluation against the full pseudo-spectral RHS
    modes, coefs = inputs.sparse_modes(n, seed=n, count=10)
    uh = inputs.sparse_to_half_spectrum(n, modes, coefs)
    prm = orc.Params(eps=3e-3, m_cut=2.5)
    full = orc.rhs(uh, n, prm)
    K = orc.kcut(n)
    ks = np.arange(-K, K + 1)
    outm = np.array([(a, b, c) for a in range(0, K + 1) for b in ks for c in ks])
    got = orc.rhs_sparse(modes, coefs, outm, n, prm)
    ref = np.stack([full[:, c % n, b % n, a] for a, b, c in outm])
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(ref)) > 1e-3


# ---------------------------------------------------------------- div_rel
# div_rel = ||(I - P) u-hat|| / ||u-hat|| (the relative size of the part the
# Leray projection of eq. (2.5) removes).  Pinned on fields whose longitudinal
# and transversal parts are known in physical space, so the expected values
# come from grid means (Parseval) and not from the oracle's spectral formula.
def _gradient_field(n):
    # u = grad phi, phi = sin(2x + y) + cos(z - 3y): purely longitudinal
    x, y, z = inputs.grid(n)
    return np.stack([2 * np.cos(2 * x + y), np.cos(2 * x + y) + 3 * np.sin(z - 3 * y), -np.sin(z - 3 * y)])


@pytest.mark.parametrize("n", [12, 16])
def test_div_rel_of_a_gradient_is_one(orc, n):
    g = _gradient_field(n)
    assert abs(orc.div_rel(inputs.half_spectrum(g), n) - 1.0) <= 1e-14


@pytest.mark.parametrize("a", [0.3, 1.0, 2.5])
def test_div_rel_of_solenoidal_plus_gradient(orc, a):
    # Taylor-Green is divergence-free and L2-orthogonal to any gradient on the
    # torus, so ||(I-P)(s + a g)||^2 = a^2 mean|g|^2 and ||s + a g||^2 =
    # mean|s|^2 + a^2 mean|g|^2
    n = 16
    s = inputs.taylor_green(n)
    g = _gradient_field(n)
    es = np.mean(np.sum(s * s, axis=0))
    eg = np.mean(np.sum(g * g, axis=0))
    want = np.sqrt(a * a * eg / (es + a * a * eg))
    assert abs(orc.div_rel(inputs.half_spectrum(s + a * g), n) - want) <= 1e-14


def test_div_rel_counts_the_mean_flow_in_the_norm_only(orc):
    # a constant flow is divergence-free (k = 0 has no longitudinal part) but
    # belongs to ||u||: u = c + g gives sqrt(mean|g|^2 / (|c|^2 + mean|g|^2))
    n = 12
    g = _gradient_field(n)
    c = np.array([0.7, -0.2, 1.1])
    u = g + c[:, None, None, None]
    eg = np.mean(np.sum(g * g, axis=0))
    want = np.sqrt(eg / (np.dot(c, c) + eg))
    assert abs(orc.div_rel(inputs.half_spectrum(u), n) - want) <= 1e-14


@pytest.mark.parametrize("theta", [0.0, 0.4, 1.1, np.pi / 2])
def test_div_rel_of_one_plane_wave_is_the_angle_cosine(orc, theta):
    # u = v cos(k.x) with |v| = 1 at angle theta to k: the longitudinal part
    # is (v.k/|k|) k/|k| cos(k.x), so div_rel = |cos theta|, for any k
    n = 16
    x, y, z = inputs.grid(n)
    k = np.array([2.0, -1.0, 3.0])
    kh = k / np.linalg.norm(k)
    e = np.cross(kh, [1.0, 0.0, 0.0])
    e /= np.linalg.norm(e)
    v = np.cos(theta) * kh + np.sin(theta) * e
    u = v[:, None, None, None] * np.cos(k[0] * x + k[1] * y + k[2] * z)[None]
    assert abs(orc.div_rel(inputs.half_spectrum(u), n) - abs(np.cos(theta))) <= 1e-14
