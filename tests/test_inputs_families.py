"""Pins of the generators of the paper's initial-data families (Sec. 6):
the perturbed Taylor-Green vortex (eqs. (6.1)-(6.3)) and the cylindrical
shear flow (eqs. (6.4)-(6.5)), against what their formulas fix: the Fourier
content of the first-order harmonics, symmetry and geometry of the cylinder."""
import numpy as np
import pytest

from paper_2401_09843_amd import inputs


def test_taylor_green_base_and_perturbation_spectrum():
    n = 16
    u, delta = inputs.perturbed_taylor_green(n, seed=3)
    X, Y, Z = inputs.grid(n)  # the box [0, 2 pi): X = 2 pi x
    base = np.stack([np.cos(X) * np.sin(Y) * np.sin(Z), -np.sin(X) * np.cos(Y) * np.sin(Z), 0 * X])
    eps = u - base
    k1 = np.fft.fftfreq(n, 1.0 / n).astype(int)
    # sin(2X) = (e^{2iX} - e^{-2iX}) / 2i, cos(2X) = (e^{2iX} + e^{-2iX}) / 2: the coefficient at
    # (sx, sy, sz) * 2 is 1/8 sum_ijk delta_ijk c_i(sx) c_j(sy) c_k(sz)
    c = lambda i, s: (s / 2j) if i == 0 else 0.5
    signs = [(sx, sy, sz) for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]
    A = np.array([[c(i, sx) * c(j, sy) * c(k, sz) / 8 for i in (0, 1) for j in (0, 1) for k in (0, 1)]
                  for (sx, sy, sz) in signs])
    for d in range(3):
        F = np.fft.fftn(eps[d]) / n ** 3  # [kz][ky][kx]
        b = np.array([F[(2 * sz) % n, (2 * sy) % n, (2 * sx) % n] for (sx, sy, sz) in signs])
        got = np.linalg.solve(A, b)
        assert np.max(np.abs(got - delta[d].reshape(-1))) <= 1e-15
        # nothing outside k in {+-2}^3
        mask = np.ones_like(F, dtype=bool)
        for (sx, sy, sz) in signs:
            mask[(2 * sz) % n, (2 * sy) % n, (2 * sx) % n] = False
        assert np.max(np.abs(F[mask])) <= 1e-16
    assert np.all(np.abs(delta) <= 0.025)
    # the draw order: one array [d][i][j][k]
    assert np.array_equal(delta, np.random.default_rng(3).uniform(-0.025, 0.025, size=(3, 2, 2, 2)))


def test_taylor_green_base_is_divergence_free():
    n = 16
    u, _ = inputs.perturbed_taylor_green(n, seed=0, amp=0.0)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    div = kx * np.fft.fftn(u[0]) + ky * np.fft.fftn(u[1]) + kz * np.fft.fftn(u[2])
    assert np.max(np.abs(div)) / n ** 3 <= 1e-15


def test_cylinder_without_perturbation():
    n = 64
    u, _ = inputs.cylindrical_shear(n, seed=0, delta=0.0)
    assert np.all(u[1] == 0) and np.all(u[2] == 0)
    assert np.all(u[0] == u[0][:, :, :1])  # independent of x
    # the disk's symmetries map grid points to grid points: y <-> z and (y, z) -> (1 - y, 1 - z)
    j = np.arange(n)
    plane = u[0][:, :, 0]
    assert np.array_equal(plane, plane.T)  # symmetric under y <-> z
    assert np.array_equal(plane, plane[(-j) % n][:, (-j) % n])  # under (y, z) -> (1 - y, 1 - z)
    frac = np.mean(plane < 0)
    assert abs(frac - np.pi / 16) <= 0.01
    # smooth profile: |u| <= 1 and the same sign as the sharp one away from the interface
    us, _ = inputs.cylindrical_shear(n, seed=0, delta=0.0, rho=0.05)
    assert np.all(np.abs(us[0]) <= 1)
    x, y, z = inputs.unit_grid(n)
    r = np.sqrt((y - 0.5) ** 2 + (z - 0.5) ** 2)
    far = np.abs(r - 0.25) > 0.05
    assert np.all(np.sign(us[0][far]) == u[0][far])


def test_cylinder_axis_follows_the_perturbation():
    n, seed, p, delta = 64, 5, 10, 0.025
    u, (ay, az, by, bz) = inputs.cylindrical_shear(n, seed=seed, p=p, delta=delta)
    rng = np.random.default_rng(seed)
    assert np.array_equal(ay, rng.uniform(0, 1, p)) and np.array_equal(az, rng.uniform(0, 1, p))
    assert np.array_equal(by, rng.uniform(0, 2 * np.pi, p)) and np.array_equal(bz, rng.uniform(0, 2 * np.pi, p))
    x = np.arange(n) / n
    k = np.arange(1, p + 1)
    sy = delta * np.sin(2 * np.pi * np.outer(x, k) - by) @ ay
    sz = delta * np.sin(2 * np.pi * np.outer(x, k) - bz) @ az
    g = np.arange(n) / n
    for ix in range(0, n, 7):
        inside = u[0][:, :, ix] < 0  # [z][y]
        cz = np.mean(np.nonzero(inside)[0]) / n
        cy = np.mean(np.nonzero(inside)[1]) / n
        assert abs(cy - (0.5 - sy[ix])) <= 2e-3 and abs(cz - (0.5 - sz[ix])) <= 2e-3, ix
    assert np.max(np.abs(sy)) > 0.01  # the perturbation is there
