"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws and tabulates input fields on the grid; it contains
none of the solver's arithmetic (no truncation, projection, right-hand side
or time stepping).  Both the GPU path and the CPU oracle receive the arrays
made here.

Fields are physical real arrays u[3][z][y][x] on the grid x_j = 2*pi*j/N of
the periodic box [0, 2*pi]^3.
"""
from __future__ import annotations

import numpy as np


def grid(n: int):
    x = 2.0 * np.pi * np.arange(n) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    return xx, y, z


def taylor_green(n: int) -> np.ndarray:
    """u = (sin x cos y cos z, -cos x sin y cos z, 0)."""
    x, y, z = grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(x) * np.cos(y) * np.cos(z)
    u[1] = -np.cos(x) * np.sin(y) * np.cos(z)
    return u


def taylor_green_2d(n: int) -> np.ndarray:
    """The z-independent field (sin x cos y, -cos x sin y, 0)."""
    x, y, z = grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(x) * np.cos(y)
    u[1] = -np.cos(x) * np.sin(y)
    return u


def abc_flow(n: int, k0: int = 1, A: float = 1.0, B: float = 1.0, C: float = 1.0) -> np.ndarray:
    """Arnold-Beltrami-Childress field at wavenumber k0 (curl u = k0 u)."""
    x, y, z = grid(n)
    u = np.empty((3, n, n, n))
    u[0] = A * np.sin(k0 * z) + C * np.cos(k0 * y)
    u[1] = B * np.sin(k0 * x) + A * np.cos(k0 * z)
    u[2] = C * np.sin(k0 * y) + B * np.cos(k0 * x)
    return u


def helical_mode(n: int, k=(7, 7, 7), amp: float = 1.0, phase: float = 0.3) -> np.ndarray:
    """Single helical (Beltrami) Fourier mode: u = Re[h exp(i k.x + i phase)]
    with h = a + i (k/|k|) x a, a a unit vector orthogonal to k, so that
    curl u = |k| u and the nonlinear term is a pure gradient."""
    kv = np.asarray(k, dtype=np.float64)
    kn = kv / np.linalg.norm(kv)
    t = np.array([1.0, 0.0, 0.0]) if abs(kn[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    a = np.cross(kn, t)
    a /= np.linalg.norm(a)
    b = np.cross(kn, a)
    x, y, z = grid(n)
    th = kv[0] * x + kv[1] * y + kv[2] * z + phase
    u = np.empty((3, n, n, n))
    for c in range(3):
        u[c] = amp * (a[c] * np.cos(th) - b[c] * np.sin(th))
    return u


def shear_profile(y: np.ndarray, rho: float) -> np.ndarray:
    """Doubly periodic shear layer: tanh((y-pi/2)/rho) for y < pi and
    tanh((3pi/2-y)/rho) for y >= pi."""
    return np.where(y < np.pi, np.tanh((y - np.pi / 2) / rho), np.tanh((1.5 * np.pi - y) / rho))


def draw_modes(rng: np.random.Generator, nmodes: int = 16, kmax: float = 4.0):
    """nmodes random Fourier modes: wave vector k uniform over the integer
    vectors with 0 < |k| <= kmax, unit amplitude vector a orthogonal to k
    (uniform angle), phase uniform in [0, 2 pi)."""
    r = int(np.floor(kmax))
    cand = np.array([(i, j, l) for i in range(-r, r + 1) for j in range(-r, r + 1) for l in range(-r, r + 1)
                     if 0 < i * i + j * j + l * l <= kmax * kmax], dtype=np.int64)
    modes = []
    for _ in range(nmodes):
        k = cand[rng.integers(len(cand))]
        kn = k / np.linalg.norm(k)
        t = np.array([1.0, 0.0, 0.0]) if abs(kn[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(kn, t)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(kn, e1)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        a = np.cos(ang) * e1 + np.sin(ang) * e2
        phi = rng.uniform(0.0, 2.0 * np.pi)
        modes.append((k.copy(), a, phi))
    return modes


def shear_layer(n: int, seed: int = 0, rho: float = 0.05, delta=0.025, nmodes: int = 16, kmax: float = 4.0):
    """Seeded perturbed doubly periodic shear layer.

    delta is a number, or a (lo, hi) pair from which delta is drawn uniformly
    first from the sample's stream.  Returns (u, delta, modes); u is not
    projected (the solver's initial projection does that)."""
    rng = np.random.default_rng(seed)
    if isinstance(delta, (tuple, list)):
        delta = float(rng.uniform(delta[0], delta[1]))
    modes = draw_modes(rng, nmodes, kmax)
    x, y, z = grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = shear_profile(y, rho)
    for k, a, phi in modes:
        th = k[0] * x + k[1] * y + k[2] * z + phi
        c = np.cos(th)
        for comp in range(3):
            u[comp] += delta * a[comp] * c
    return u, float(delta), modes


def unit_grid(n: int):
    """Coordinates of the grid on the unit torus used by the paper's
    initial-data families (x = X / 2 pi for this box's X in [0, 2 pi))."""
    x = np.arange(n) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    return xx, y, z


def perturbed_taylor_green(n: int, seed: int = 0, amp: float = 0.025):
    """The perturbed Taylor-Green vortex of Sec. 6.1 (eqs. (6.1)-(6.3)) on
    the unit torus: u = cos(2 pi x) sin(2 pi y) sin(2 pi z) + eps_0,
    v = -sin(2 pi x) cos(2 pi y) sin(2 pi z) + eps_1, w = eps_2, with
    eps_d = 1/8 sum over (i,j,k) in {0,1}^3 of delta_{d,i,j,k}
    alpha_i(4 pi x) alpha_j(4 pi y) alpha_k(4 pi z), alpha_0 = sin,
    alpha_1 = cos, and the 24 amplitudes delta ~ U[-amp, amp] i.i.d., drawn
    as one array [d][i][j][k] from default_rng(seed).  Returns (u, delta)."""
    rng = np.random.default_rng(seed)
    delta = rng.uniform(-amp, amp, size=(3, 2, 2, 2))
    x, y, z = unit_grid(n)
    tp = 2.0 * np.pi
    u = np.zeros((3, n, n, n))
    u[0] = np.cos(tp * x) * np.sin(tp * y) * np.sin(tp * z)
    u[1] = -np.sin(tp * x) * np.cos(tp * y) * np.sin(tp * z)
    alpha = lambda i, t: np.sin(t) if i == 0 else np.cos(t)
    for d in range(3):
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    u[d] += delta[d, i, j, k] / 8.0 * alpha(i, 2 * tp * x) * alpha(j, 2 * tp * y) * alpha(k, 2 * tp * z)
    return u, delta


def cylindrical_shear(n: int, seed: int = 0, rho: float = 0.0, p: int = 10, delta: float = 0.025):
    """The cylindrical shear flow of Sec. 6.2 (eqs. (6.4)-(6.5)) on the unit
    torus: u = tanh(2 pi (r - 1/4) / rho) (for rho = 0: -1 where r <= 1/4,
    else 1), v = w = 0, with r^2 = (y - 1/2 + s_y(x))^2 + (z - 1/2 + s_z(x))^2
    and s_c(x) = delta sum_{k=1..p} a_k^c sin(2 pi k x - b_k^c), a ~ U[0,1],
    b ~ U[0, 2 pi], drawn from default_rng(seed) in the order a^y, a^z, b^y,
    b^z (p values each).  Returns (u, (a_y, a_z, b_y, b_z))."""
    rng = np.random.default_rng(seed)
    ay, az = rng.uniform(0.0, 1.0, p), rng.uniform(0.0, 1.0, p)
    by, bz = rng.uniform(0.0, 2.0 * np.pi, p), rng.uniform(0.0, 2.0 * np.pi, p)
    x, y, z = unit_grid(n)
    xs = x[0, 0, :]
    k = np.arange(1, p + 1)
    sy = delta * np.sum(ay[:, None] * np.sin(2 * np.pi * k[:, None] * xs[None, :] - by[:, None]), axis=0)
    sz = delta * np.sum(az[:, None] * np.sin(2 * np.pi * k[:, None] * xs[None, :] - bz[:, None]), axis=0)
    r = np.sqrt((y - 0.5 + sy[None, None, :]) ** 2 + (z - 0.5 + sz[None, None, :]) ** 2)
    u = np.zeros((3, n, n, n))
    u[0] = np.where(r <= 0.25, -1.0, 1.0) if rho == 0 else np.tanh(2 * np.pi * (r - 0.25) / rho)
    return u, (ay, az, by, bz)


def cfl_dt(u: np.ndarray, cfl: float = 0.5) -> float:
    """dt = cfl * (2 pi / N) / max_x(|u|+|v|+|w|) of the given field."""
    n = u.shape[-1]
    return float(cfl * (2.0 * np.pi / n) / np.max(np.abs(u).sum(axis=0)))


def random_field(n: int, seed: int, slope: float = 1.0, ncomp: int = 3) -> np.ndarray:
    """Seeded random real field with a decaying spectrum: Gaussian modes
    weighted by (1 + |k|^2)^(-slope/2), tabulated on the grid."""
    rng = np.random.default_rng(seed)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    w = (1.0 + kx * kx + ky * ky + kz * kz) ** (-slope / 2.0)
    spec = (rng.standard_normal((ncomp, n, n, n)) + 1j * rng.standard_normal((ncomp, n, n, n))) * w
    u = np.fft.ifftn(spec, axes=(-3, -2, -1)).real
    return u / np.sqrt(np.mean(u * u))


def half_spectrum(u: np.ndarray) -> np.ndarray:
    """numpy's normalised half spectrum of a real field (the solver's public
    layout): rfftn(u, norm="forward") over the last three axes."""
    return np.fft.rfftn(u, axes=(-3, -2, -1), norm="forward")


def shear_layer_torch(n: int, seed: int = 0, rho: float = 0.05, delta=0.025, nmodes: int = 16, kmax: float = 4.0,
                      device="cuda", dtype=None):
    """The field of shear_layer(n, seed, ...) tabulated with torch on a
    device (same random draws, same formula), for grids too large for the
    host.  Returns (u, delta, modes) with u a torch tensor [3, n, n, n]."""
    import torch

    dtype = dtype or torch.float64
    rng = np.random.default_rng(seed)
    if isinstance(delta, (tuple, list)):
        delta = float(rng.uniform(delta[0], delta[1]))
    modes = draw_modes(rng, nmodes, kmax)
    x1 = 2.0 * np.pi * torch.arange(n, device=device, dtype=torch.float64) / n
    X = x1.view(1, 1, n)
    Y = x1.view(1, n, 1)
    Z = x1.view(n, 1, 1)
    u = torch.zeros((3, n, n, n), device=device, dtype=dtype)
    prof = torch.where(x1 < np.pi, torch.tanh((x1 - np.pi / 2) / rho), torch.tanh((1.5 * np.pi - x1) / rho))
    u[0] += prof.view(1, n, 1).to(dtype)
    for k, a, phi in modes:
        c = torch.cos(float(k[0]) * X + float(k[1]) * Y + float(k[2]) * Z + float(phi)).to(dtype)
        for comp in range(3):
            if a[comp] != 0.0:
                u[comp].add_(c, alpha=float(delta * a[comp]))
        del c
    return u, float(delta), modes


def sparse_modes(n: int, seed: int, count: int = 24, kmax=None):
    """A seeded real field with a sparse spectrum: `count` random wave
    vectors in the cube |k_i| <= kmax (default the 2/3 cutoff floor((N-1)/3),
    edges included) with k_x >= 0, random complex amplitudes, plus the
    conjugate partner of each.  Returns (modes int [m,3] as (kx,ky,kz),
    coefs complex [m,3]) listing the full spectrum."""
    K = (n - 1) // 3 if kmax is None else kmax
    rng = np.random.default_rng(seed)
    chosen = {}
    edges = [K, -K, K - 1, 1, 0]
    while len(chosen) < count:
        if len(chosen) < 6:  # some modes on the cutoff edges
            k = (int(rng.choice([K, K - 1, 1])), int(rng.choice(edges)), int(rng.choice(edges)))
        else:
            k = (int(rng.integers(0, K + 1)), int(rng.integers(-K, K + 1)), int(rng.integers(-K, K + 1)))
        if k == (0, 0, 0):
            continue
        if k[0] == 0 and (-k[0], -k[1], -k[2]) in chosen:
            continue
        chosen[k] = (rng.standard_normal(3) + 1j * rng.standard_normal(3)) / np.sqrt(2 * count)
    modes, coefs = [], []
    for k, c in chosen.items():
        modes.append(k)
        coefs.append(c)
        modes.append((-k[0], -k[1], -k[2]))
        coefs.append(np.conj(c))
    return np.array(modes, dtype=np.int64), np.array(coefs)


def sparse_to_half_spectrum(n: int, modes: np.ndarray, coefs: np.ndarray) -> np.ndarray:
    """Scatter a sparse full spectrum into the half-spectrum layout
    [3][N][N][N/2+1] (entries with k_x >= 0 only)."""
    h = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    for (kx, ky, kz), c in zip(modes, coefs):
        if kx >= 0:
            h[:, kz % n, ky % n, kx] = c
    return h
