"""Discrete adjoint on the GPU: the adjoint SSP-RK3 step against the
oracle's, the tape path against the recompute path, and the differentiable
rollout against the oracle's reference gradient and central differences."""
import time

import numpy as np
import pytest
import torch

from paper_2401_09843_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_2401_09843_amd import ns as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _cube(n):
    K = (n - 1) // 3
    k = np.abs(np.fft.fftfreq(n, 1.0 / n))
    kx = np.arange(n // 2 + 1)
    return ((k[:, None, None] <= K) & (k[None, :, None] <= K) & (kx[None, None, :] <= K))[None]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cuda(a, dtype=torch.float64):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if np.iscomplexobj(a):
        t = t.to(torch.complex128 if dtype == torch.float64 else torch.complex64)
    else:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
@pytest.mark.parametrize("n", [16, 24, 32, 48, 64])
def test_adjoint_step_matches_oracle(ns, orc, n, dtype, tol):
    print("adjoint step n=%d %s" % (n, dtype), flush=True)
    prm = orc.Params(eps=3e-3, m_cut=2.0)
    u = inputs.random_field(n, seed=700 + n)
    uh = orc.initial_state(u, prm)
    dt = 0.5 * inputs.cfl_dt(u)
    # lambda supported in the 2/3 cube: the library's step ignores modes
    # outside it (they are outputs of zero), the oracle's carries them
    lam = orc.project(inputs.half_spectrum(inputs.random_field(n, seed=800 + n)), n, orc.Params(eps=0.0))
    lam = lam + 0.3 * orc.forward(inputs.random_field(n, seed=900 + n)) * _cube(n)
    ref = orc.adjoint_step(uh, lam, n, dt, prm)
    S = ns.Solver(n, dtype=dtype, eps=3e-3, m_cut=2.0, graph=False)
    # recompute path
    l1 = cuda(lam, dtype)
    S.adjoint_step(l1, dt, uhat_n=cuda(uh, dtype))
    assert rel(l1.cpu().numpy(), ref) <= tol
    # tape path: the forward step is taped, then the adjoint reads it
    x = cuda(uh, dtype)
    tape = S.new_tape(1)
    S.step_taped(x, dt, 1, tape)
    l2 = cuda(lam, dtype)
    S.adjoint_step(l2, dt, tape=tape, step=0)
    assert torch.equal(l1, l2)
    # and the taped step equals the plain step
    y = cuda(uh, dtype)
    S.step(y, dt, 1)
    assert torch.equal(x, y)


def shell_weight(n, lo, hi, device="cuda"):
    k1 = torch.fft.fftfreq(n, 1.0 / n, device=device, dtype=torch.float64)
    kz, ky, kx = torch.meshgrid(k1, k1, torch.arange(n // 2 + 1, device=device, dtype=torch.float64), indexing="ij")
    kk = torch.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    return ((kk >= lo) & (kk < hi)).to(torch.float64)


def shell_energy(u, w):
    """J = 1/2 sum over the full spectrum of w |u-hat|^2 from the half
    spectrum (modes with 0 < k_x < N/2 count twice)."""
    n = u.shape[-1]
    uh = torch.fft.rfftn(u, dim=(-3, -2, -1), norm="forward")
    mult = torch.full((n // 2 + 1,), 2.0, dtype=torch.float64, device=u.device)
    mult[0] = 1.0
    mult[-1] = 1.0
    return 0.5 * torch.sum(w * mult * uh.real ** 2 + w * mult * uh.imag ** 2)


def test_rollout_gradient_matches_oracle(ns, orc):
    n, steps = 32, 40
    u0 = inputs.shear_layer(n, seed=0, rho=0.15)[0]
    dt = inputs.cfl_dt(u0)
    prm = orc.Params(eps=1e-3)
    w = shell_weight(n, 4, 8)
    J_ref, g_ref = orc.rollout_gradient(u0, dt, steps, w.cpu().numpy(), prm)
    S = ns.Solver(n, dtype=torch.float64, eps=1e-3)
    x = cuda(u0).requires_grad_(True)
    uT = ns.rollout(x, S, dt, steps, ckpt_every=15)
    J = shell_energy(uT, w)
    J.backward()
    assert abs(J.item() - J_ref) <= 1e-11 * abs(J_ref)
    assert rel(x.grad.cpu().numpy(), g_ref) <= 1e-10


def test_rollout_gradient_finite_differences_128(ns):
    """128^3 FP64, 200 steps, checkpoints every 20: <grad, v> against
    central differences (eps = 1e-6) on 8 seeded directions."""
    n, steps = 128, 200
    u0, _, _ = inputs.shear_layer_torch(n, seed=0, device="cuda")
    dt = float(0.5 * (2 * np.pi / n) / u0.abs().sum(0).max().item())
    w = shell_weight(n, 8, 16)
    S = ns.Solver(n, dtype=torch.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        uh = S.forward(u0)
        S.step(uh, dt, steps)
        J0 = shell_energy(S.inverse(uh), w).item()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    x = u0.clone().requires_grad_(True)
    t0 = time.perf_counter()
    J = shell_energy(ns.rollout(x, S, dt, steps, ckpt_every=20), w)
    J.backward()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    assert abs(J.item() - J0) <= 1e-12 * abs(J0)
    print("128^3 200 steps: forward %.3f s, forward+backward %.3f s, ratio %.2f" % (t_fwd, t_fb, t_fb / t_fwd),
          flush=True)
    g = x.grad
    rms = u0.pow(2).mean().sqrt()
    worst = 0.0
    for seed in range(2000, 2008):
        gen = torch.Generator(device="cuda").manual_seed(seed)
        v = torch.randn(u0.shape, generator=gen, device="cuda", dtype=torch.float64)
        v *= rms / v.pow(2).mean().sqrt()
        eps = 1e-6
        with torch.no_grad():
            Jp = S.forward(u0 + eps * v)
            S.step(Jp, dt, steps)
            Jp = shell_energy(S.inverse(Jp), w).item()
            Jm = S.forward(u0 - eps * v)
            S.step(Jm, dt, steps)
            Jm = shell_energy(S.inverse(Jm), w).item()
        fd = (Jp - Jm) / (2 * eps)
        ad = torch.sum(g * v).item()
        worst = max(worst, abs(fd - ad) / abs(fd))
        print("direction %d: fd %.12e adjoint %.12e rel %.2e" % (seed, fd, ad, abs(fd - ad) / abs(fd)), flush=True)
    assert worst <= 1e-6
