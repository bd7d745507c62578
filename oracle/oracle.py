"""Python glue for the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the solver never does.  It shares no
code with the GPU library.

Public spectra here use the half-spectrum (R2C) layout [3][N][N][N/2+1] of a
real field u[3][z][y][x], i.e. numpy.fft.rfftn(u, axes=(-3,-2,-1),
norm="forward").  The C oracle works on full complex N^3 spectra; the helpers
below only convert layouts (Hermitian extension, slicing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, OpenMP over lines)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("s", ctypes.c_double), ("m_cut", ctypes.c_double),
                ("q_kind", ctypes.c_int), ("theta", ctypes.c_double), ("kcut", ctypes.c_int)]


@dataclass
class Params:
    """Model parameters of eqs. (2.1)-(2.4).  eps/m_cut < 0 select the
    defaults eps_N = 1e-3 (32/N)^(2s-1) and m_N = N/3; kcut < 0 selects the
    2/3-rule cutoff floor((N-1)/3)."""
    eps: float = -1.0
    s: float = 1.5
    m_cut: float = -1.0
    q_kind: int = 0
    theta: float = 1.0
    kcut: int = -1

    def resolved(self, n: int) -> "Params":
        eps = self.eps if self.eps >= 0 else 1e-3 * (32.0 / n) ** (2.0 * self.s - 1.0)
        m = self.m_cut if self.m_cut >= 0 else n / 3.0
        return Params(eps, self.s, m, self.q_kind, self.theta, self.kcut)

    def c(self, n: int) -> _Params:
        r = self.resolved(n)
        return _Params(r.eps, r.s, r.m_cut, r.q_kind, r.theta, r.kcut)


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        pp = ctypes.POINTER(_Params)
        sig = {
            "orc_dft1": (None, [I, P, P, I]),
            "orc_fft3": (None, [I, P, I]),
            "orc_dft3_brute": (None, [I, P, P, I]),
            "orc_project": (None, [I, pp, P]),
            "orc_forward": (None, [I, P, P]),
            "orc_inverse": (D, [I, I, P, P]),
            "orc_rhs": (D, [I, pp, P, P]),
            "orc_ssprk3": (None, [I, pp, P, D, I]),
            "orc_rhs_vjp": (None, [I, pp, P, P, P]),
            "orc_adjoint_step": (None, [I, pp, P, D, P]),
            "orc_energy_spectrum": (None, [I, P, P, I]),
            "orc_div_rel": (D, [I, P]),
            "orc_rhs_sparse": (None, [pp, I, P, P, I, P, P]),
            "orc_num_threads": (I, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- layouts
def full_from_r2c(h: np.ndarray, n: int) -> np.ndarray:
    """Hermitian extension of a half spectrum [..., N, N, N/2+1] to the full
    [..., N, N, N] spectrum: X[kz,ky,kx] = conj(X[-kz,-ky,-kx]) for kx > N/2."""
    h = np.asarray(h, dtype=np.complex128)
    out = np.zeros(h.shape[:-1] + (n,), dtype=np.complex128)
    nh = n // 2 + 1
    out[..., :nh] = h
    iz = (-np.arange(n)) % n
    for kx in range(nh, n):
        plane = h[..., :, :, n - kx]
        out[..., kx] = np.conj(plane[..., iz, :][..., :, iz])
    return np.ascontiguousarray(out)


def r2c_from_full(f: np.ndarray, n: int) -> np.ndarray:
    return np.ascontiguousarray(f[..., : n // 2 + 1])


# ---------------------------------------------------------------- transforms
def dft1(x: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised 1-D DFT by the oracle's recursive mixed-radix routine."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    lib().orc_dft1(x.size, _ptr(x), _ptr(out), sign)
    return out


def fft3(a: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised 3-D DFT of an N^3 complex array (recursive, per axis)."""
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    lib().orc_fft3(a.shape[0], _ptr(a), sign)
    return a


def dft3_brute(a: np.ndarray, sign: int) -> np.ndarray:
    """The 3-D DFT summed from its definition, O(N^6)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    out = np.empty_like(a)
    lib().orc_dft3_brute(a.shape[0], _ptr(a), _ptr(out), sign)
    return out


def forward(u: np.ndarray) -> np.ndarray:
    """Physical real [3][N]^3 -> normalised half spectrum (no truncation)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.shape[-1]
    full = np.empty(u.shape, dtype=np.complex128)
    lib().orc_forward(n, _ptr(u), _ptr(full))
    return r2c_from_full(full, n)


def inverse(uh: np.ndarray, n: int) -> np.ndarray:
    """Half spectrum [c][N][N][N/2+1] -> physical real [c][N]^3."""
    full = full_from_r2c(uh, n)
    nc = full.shape[0]
    u = np.empty((nc, n, n, n), dtype=np.float64)
    lib().orc_inverse(n, nc, _ptr(full), _ptr(u))
    return u


# ---------------------------------------------------------------- the method
def project(uh: np.ndarray, n: int, prm: Params = Params()) -> np.ndarray:
    """T P u-hat: 2/3 truncation and Leray projection."""
    full = full_from_r2c(uh, n)
    c = prm.c(n)
    lib().orc_project(n, ctypes.byref(c), _ptr(full))
    return r2c_from_full(full, n)


def initial_state(u0: np.ndarray, prm: Params = Params()) -> np.ndarray:
    """u-hat(0) = T P F[u0] from a physical field (eq. (2.1), third line)."""
    n = u0.shape[-1]
    return project(forward(u0), n, prm)


def rhs(uh: np.ndarray, n: int, prm: Params = Params()) -> np.ndarray:
    """One evaluation of the SHV right-hand side F(u-hat)."""
    full = full_from_r2c(uh, n)
    out = np.empty_like(full)
    c = prm.c(n)
    lib().orc_rhs(n, ctypes.byref(c), _ptr(full), _ptr(out))
    return r2c_from_full(out, n)


def ssprk3(uh: np.ndarray, n: int, dt: float, nsteps: int, prm: Params = Params()) -> np.ndarray:
    full = full_from_r2c(uh, n)
    c = prm.c(n)
    lib().orc_ssprk3(n, ctypes.byref(c), _ptr(full), float(dt), int(nsteps))
    return r2c_from_full(full, n)


def rhs_vjp(uh: np.ndarray, lam: np.ndarray, n: int, prm: Params = Params()) -> np.ndarray:
    """F'(u-hat)^T lambda in the full-spectrum inner product Re sum conj(a) b."""
    fu = full_from_r2c(uh, n)
    fl = full_from_r2c(lam, n)
    out = np.empty_like(fu)
    c = prm.c(n)
    lib().orc_rhs_vjp(n, ctypes.byref(c), _ptr(fu), _ptr(fl), _ptr(out))
    return r2c_from_full(out, n)


def adjoint_step(uh: np.ndarray, lam: np.ndarray, n: int, dt: float, prm: Params = Params()) -> np.ndarray:
    """dJ/du^{n+1} -> dJ/du^n through one SSP-RK3 step taken from u^n = uh."""
    fu = full_from_r2c(uh, n)
    fl = full_from_r2c(lam, n)
    c = prm.c(n)
    lib().orc_adjoint_step(n, ctypes.byref(c), _ptr(fu), float(dt), _ptr(fl))
    return r2c_from_full(fl, n)


def energy_spectrum(uh: np.ndarray, n: int, nbins: int) -> np.ndarray:
    full = full_from_r2c(uh, n)
    E = np.zeros(nbins, dtype=np.float64)
    lib().orc_energy_spectrum(n, _ptr(full), _ptr(E), nbins)
    return E


def enstrophy_spectrum(uh: np.ndarray, n: int, nbins: int) -> np.ndarray:
    """Z(kappa) = 1/2 sum over the full spectrum of |k x u-hat_k|^2 for
    round(|k|) = kappa (the enstrophy-spectrum writer of Sec. 2.4; the
    vorticity is i k x u-hat)."""
    full = full_from_r2c(uh, n)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    wx = ky * full[2] - kz * full[1]
    wy = kz * full[0] - kx * full[2]
    wz = kx * full[1] - ky * full[0]
    dens = 0.5 * (np.abs(wx) ** 2 + np.abs(wy) ** 2 + np.abs(wz) ** 2)
    shell = np.rint(np.sqrt(kx * kx + ky * ky + kz * kz)).astype(np.int64)
    Z = np.zeros(nbins)
    ok = shell < nbins
    np.add.at(Z, shell[ok], dens[ok])
    return Z


def moments(uhs, n: int):
    """Pointwise mean and variance of the empirical measure of Algorithm 1
    over samples u_b = F^-1[u-hat_b] (half spectra of one size n):
    mean = (1/B) sum_b u_b, var = (1/B) sum_b (u_b - mean)^2."""
    us = [inverse(uh, n) for uh in uhs]
    mean = sum(us) / len(us)
    var = sum((u - mean) ** 2 for u in us) / len(us)
    return mean, var


def structure_functions(uh: np.ndarray, n: int, lmax: int, p: float) -> np.ndarray:
    """Longitudinal velocity structure functions of order p (the structure-
    function writers of Sec. 2.4; reading: increments of each component
    along its own axis, averaged over the three axes):
    S_p(l) = 1/3 sum_d mean_x |u_d(x + l h e_d) - u_d(x)|^p, h = 2 pi / n,
    l = 1..lmax, for u = F^-1[u-hat] on the n grid."""
    u = inverse(uh, n)  # [c][z][y][x]
    axis = {0: 2, 1: 1, 2: 0}  # component d varies along array axis
    S = np.zeros(lmax)
    for l in range(1, lmax + 1):
        S[l - 1] = sum(np.mean(np.abs(np.roll(u[d], -l, axis=axis[d]) - u[d]) ** p) for d in range(3)) / 3.0
    return S


def wasserstein1_pointwise(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """1-D Wasserstein-1 distance between the empirical distributions of
    a[:, i] (na samples) and b[:, i] (nb samples) at every position i:
    W1 = integral over t of |F_a(t) - F_b(t)|, with F the empirical CDFs,
    summed exactly between the merged sample values."""
    a = np.sort(np.asarray(a, dtype=np.float64), axis=0)
    b = np.sort(np.asarray(b, dtype=np.float64), axis=0)
    na, nb = a.shape[0], b.shape[0]
    t = np.sort(np.concatenate([a, b], axis=0), axis=0)  # breakpoints
    out = np.zeros(a.shape[1:])
    for j in range(na + nb - 1):
        lo = t[j]
        # F at the interval (t_j, t_{j+1}): the fraction of samples <= t_j
        Fa = np.sum(a <= lo[None], axis=0) / na
        Fb = np.sum(b <= lo[None], axis=0) / nb
        out += np.abs(Fa - Fb) * (t[j + 1] - lo)
    return out


def wasserstein1_fields(ua: np.ndarray, ub: np.ndarray):
    """The 1-point marginal distance between two ensembles of physical fields
    ua [na][3][N][N][N] and ub [nb][3][N][N][N]: W1 of each component's
    marginal at each point (reading: component by component), as a field
    [3][N][N][N], and its mean over the points per component."""
    w = wasserstein1_pointwise(ua.reshape(ua.shape[0], -1), ub.reshape(ub.shape[0], -1)).reshape(ua.shape[1:])
    return w, w.reshape(3, -1).mean(axis=1)


def div_rel(uh: np.ndarray, n: int) -> float:
    full = full_from_r2c(uh, n)
    return float(lib().orc_div_rel(n, _ptr(full)))


def num_threads() -> int:
    """Threads of the oracle's OpenMP loops."""
    return int(lib().orc_num_threads())


def kcut(n: int) -> int:
    return (n - 1) // 3


def rhs_sparse(modes: np.ndarray, coefs: np.ndarray, out_modes: np.ndarray, n: int, prm: Params = Params()):
    """F at out_modes for a field whose full spectrum is nonzero only at
    `modes` (int [m,3] as (kx,ky,kz), including the conjugate of every mode)
    with coefficients coefs (complex [m,3]).  Galerkin triad sum."""
    kin = np.ascontiguousarray(modes, dtype=np.int32)
    uin = np.ascontiguousarray(coefs, dtype=np.complex128)
    kout = np.ascontiguousarray(out_modes, dtype=np.int32)
    out = np.zeros((len(kout), 3), dtype=np.complex128)
    c = prm.c(n)
    lib().orc_rhs_sparse(ctypes.byref(c), len(kin), _ptr(kin), _ptr(uin), len(kout), _ptr(kout), _ptr(out))
    return out


def padded_cutoff(n: int) -> int:
    """Retained wavenumbers |k_i| <= n/2 - 1 of an n-mode state: the Nyquist
    planes k_i = -n/2 of the n-point half spectrum are left out (reading of
    Algorithm 2, which does not treat them)."""
    return n // 2 - 1


def rhs_padded(uh: np.ndarray, n: int, npad: int, prm: Params = Params()) -> np.ndarray:
    """The right-hand side by Algorithm 2 as stated, for a state of n modes
    per axis (half spectrum [3][n][n][n/2+1]):
      1. pad u-hat with zeros to npad >= 3n/2 points per axis,
      2. u = F^-1[u-hat] on the padded grid,
      3. the six products B_ij = u_i u_j,
      4. B-hat = F[B],
      5. drop the frequencies the n-mode state does not hold,
      6. b = -i k.B-hat, the Leray projection (eq. (2.5)) and the
         hyperviscosity of eqs. (2.1)-(2.4), with eps/m_cut defaults taken
         at the mode resolution n.
    Retained modes: |k_i| <= padded_cutoff(n); the output is zero elsewhere.
    The transforms are numpy's FFTs (a library primitive); the spectra are
    normalised by the number of grid points, as everywhere here."""
    if 2 * npad < 3 * n:
        raise ValueError("Algorithm 2 needs npad >= 3n/2 (n=%d, npad=%d)" % (n, npad))
    K = padded_cutoff(n)
    r = prm.resolved(n)
    full = full_from_r2c(uh, n)  # [3][z][y][x]
    k = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    src = np.flatnonzero(np.abs(k) <= K)  # n-grid indices of the retained wavenumbers
    kr = k[src]
    dst = kr % npad  # the same wavenumbers on the padded grid
    # 1. pad
    P = np.zeros((3, npad, npad, npad), dtype=np.complex128)
    for c in range(3):
        P[c][np.ix_(dst, dst, dst)] = full[c][np.ix_(src, src, src)]
    # 2. inverse transform (u(x) = sum_k u-hat_k exp(i k.x))
    u = np.real(np.fft.ifftn(P, axes=(1, 2, 3))) * float(npad) ** 3
    del P
    # 3.-5. products, forward transform, keep the retained frequencies
    kz, ky, kx = np.meshgrid(kr, kr, kr, indexing="ij")
    kv = (kx.astype(np.float64), ky.astype(np.float64), kz.astype(np.float64))
    b = [np.zeros(kx.shape, dtype=np.complex128) for _ in range(3)]
    for i in range(3):
        for j in range(i, 3):
            Bh = np.fft.fftn(u[i] * u[j]) / float(npad) ** 3
            Bh = Bh[np.ix_(dst, dst, dst)]
            # 6. b_i = -i sum_j k_j B_ij, with B symmetric
            b[i] += -1j * kv[j] * Bh
            if j != i:
                b[j] += -1j * kv[i] * Bh
    del u
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    kb = kv[0] * b[0] + kv[1] * b[1] + kv[2] * b[2]
    safe = np.where(k2 > 0, k2, 1.0)
    kabs = np.sqrt(k2)
    if r.q_kind == 0:
        q = (kabs > r.m_cut).astype(np.float64)
    else:
        with np.errstate(divide="ignore"):
            q = np.where(kabs > r.m_cut, 1.0 - (r.m_cut / np.where(kabs > 0, kabs, 1.0)) ** ((2 * r.s - 1) / r.theta), 0.0)
    rate = r.eps * k2 ** r.s * q
    out = np.zeros_like(full)
    for i in range(3):
        ci = b[i] - np.where(k2 > 0, kv[i] * kb / safe, 0.0)
        out[i][np.ix_(src, src, src)] = ci - rate * full[i][np.ix_(src, src, src)]
    return r2c_from_full(out, n)


def embed_padded(uh: np.ndarray, n: int, npad: int) -> np.ndarray:
    """The retained modes of an n-mode half spectrum placed in the npad-point
    half spectrum (zero elsewhere)."""
    K = padded_cutoff(n)
    full = full_from_r2c(uh, n)
    k = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    src = np.flatnonzero(np.abs(k) <= K)
    dst = k[src] % npad
    out = np.zeros(full.shape[:-3] + (npad, npad, npad), dtype=np.complex128)
    for c in range(full.shape[0]):
        out[c][np.ix_(dst, dst, dst)] = full[c][np.ix_(src, src, src)]
    return r2c_from_full(out, npad)


def crop_padded(uh: np.ndarray, n: int, npad: int) -> np.ndarray:
    """The inverse of embed_padded: the retained modes of an npad-point half
    spectrum in the n-point half spectrum."""
    K = padded_cutoff(n)
    full = full_from_r2c(uh, npad)
    k = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    src = np.flatnonzero(np.abs(k) <= K)
    dst = k[src] % npad
    out = np.zeros(full.shape[:-3] + (n, n, n), dtype=np.complex128)
    for c in range(full.shape[0]):
        out[c][np.ix_(src, src, src)] = full[c][np.ix_(dst, dst, dst)]
    return r2c_from_full(out, n)


def rollout_gradient(u0: np.ndarray, dt: float, nsteps: int, weight: np.ndarray, prm: Params = Params()):
    """Reference gradient of J = 1/2 sum over the full spectrum of
    weight_k |u-hat_k(T)|^2 with respect to the physical u0, through
    u-hat(0) = T P F[u0] and nsteps SSP-RK3 steps; weight is a half-spectrum
    [N][N][N/2+1] real mask.  Returns (J, grad [3][N]^3)."""
    n = u0.shape[-1]
    states = [initial_state(u0, prm)]
    for _ in range(nsteps):
        states.append(ssprk3(states[-1], n, dt, 1, prm))
    uT = states[-1]
    wfull = np.real(full_from_r2c(weight[None].astype(np.complex128), n))[0]
    full = full_from_r2c(uT, n)
    J = 0.5 * float(np.sum(wfull[None] * np.abs(full) ** 2))
    lam = uT * weight[None]
    for k in range(nsteps - 1, -1, -1):
        lam = adjoint_step(states[k], lam, n, dt, prm)
    mu = project(lam, n, prm)
    return J, inverse(mu, n) / n ** 3
