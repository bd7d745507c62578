"""Algorithm 2 in its padded form on the GPU (NS_PAD): states of n modes per
axis, passes on the grid of 3n/2 points.  Against the oracle's rhs_padded
(the six steps as stated) at small n, the sparse Galerkin oracle with cutoff
n/2 - 1 at 256, 512 and 1024 modes (grids 384, 768, 1536), and the oracle's
SSP-RK3 on the padded grid for trajectories."""
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dtype):
    cd = torch.complex128 if dtype == torch.float64 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(cd).cuda()


def host(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_padded_rhs_matches_oracle(ns, orc, n, dtype, tol):
    print("padded rhs n=%d %s" % (n, dtype), flush=True)
    # the random field fills every mode of the n-point layout, Nyquist planes included
    uh = inputs.half_spectrum(inputs.random_field(n, seed=500 + n))
    ref = orc.rhs_padded(uh, n, 3 * n // 2)  # default eps / m_cut at n
    S = ns.Solver(n, dtype=dtype, graph=False, pad=True)
    got = host(S.rhs(dev(uh, dtype)))
    assert rel(got, ref) <= tol
    assert np.all(got[:, n // 2] == 0) and np.all(got[:, :, n // 2] == 0) and np.all(got[..., n // 2] == 0)


def _support(modes, K):
    s = set()
    for p in modes:
        for q in modes:
            k = p + q
            if k[0] >= 0 and np.all(np.abs(k) <= K):
                s.add(tuple(int(v) for v in k))
        if p[0] >= 0:
            s.add(tuple(int(v) for v in p))
    return np.array(sorted(s), dtype=np.int64)


@pytest.mark.parametrize("n,dtype,tol", [(256, torch.float64, 1e-12), (512, torch.float32, 1e-5),
                                         (1024, torch.float32, 1e-5)])
def test_padded_rhs_full_size_sparse(ns, orc, n, dtype, tol):
    """Sparse fields with modes on the cutoff edges |k_i| = n/2 - 1: the
    retained outputs against the triad sum, the rest of the spectrum ~ 0."""
    print("padded sparse n=%d grid %d" % (n, 3 * n // 2), flush=True)
    K = n // 2 - 1
    modes, coefs = inputs.sparse_modes(n, seed=n + 21, count=16, kmax=K)
    kout = _support(modes, K)
    ref = orc.rhs_sparse(modes, coefs, kout, n, orc.Params(kcut=K))
    cd = torch.complex128 if dtype == torch.float64 else torch.complex64
    S = ns.Solver(n, dtype=dtype, graph=False, pad=True)
    uh = torch.zeros((3, n, n, n // 2 + 1), dtype=cd, device="cuda")
    sel = modes[:, 0] >= 0
    for c in range(3):
        uh[c, torch.as_tensor(modes[sel, 2] % n), torch.as_tensor(modes[sel, 1] % n),
           torch.as_tensor(modes[sel, 0])] = torch.as_tensor(coefs[sel, c]).to(cd).cuda()
    F = S.rhs(uh)
    oz, oy, ox = (torch.as_tensor(kout[:, 2] % n), torch.as_tensor(kout[:, 1] % n), torch.as_tensor(kout[:, 0]))
    got = torch.stack([F[c, oz, oy, ox] for c in range(3)], dim=1).cpu().numpy().astype(np.complex128)

    def energy(F):  # one component at a time: at 1024 modes F is 12.9 GB
        return sum(float(torch.sum(torch.abs(F[c]).double() ** 2).item()) for c in range(3))

    total = energy(F)
    for c in range(3):
        F[c, oz, oy, ox] = 0
    off = energy(F)
    assert rel(got, ref) <= tol
    assert off <= 10 * tol ** 2 * total


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 5e-6)])
def test_padded_steps_match_oracle(ns, orc, dtype, tol, fuse):
    """10 SSP-RK3 steps of a 32-mode shear layer: the oracle steps the state
    embedded in the 48-point layout with cutoff 15 (the same method, pinned
    against rhs_padded on the CPU)."""
    n, npad, steps = 32, 48, 10
    u0, _, _ = inputs.shear_layer(n, seed=2)
    dt = inputs.cfl_dt(u0)
    uh0 = orc.initial_state(u0)
    eps, m = 1e-3, n / 3.0
    ref = orc.crop_padded(orc.ssprk3(orc.embed_padded(uh0, n, npad), npad, dt, steps,
                                     orc.Params(eps=eps, m_cut=m, kcut=orc.padded_cutoff(n))), n, npad)
    S = ns.Solver(n, dtype=dtype, pad=True, fuse=fuse)
    x = dev(uh0, dtype)
    S.step(x, dt, steps)
    assert rel(host(x), ref) <= tol


def test_padded_forward_inverse_live_on_the_padded_grid(ns, orc):
    n = 32
    S = ns.Solver(n, dtype=torch.float64, pad=True)
    u = torch.from_numpy(inputs.taylor_green(3 * n // 2)).cuda()
    uh = S.forward(u)
    assert tuple(uh.shape) == (3, n, n, n // 2 + 1)
    ref = orc.forward(inputs.taylor_green(n))  # the same modes, |k| = sqrt(3)
    assert rel(host(uh), ref) <= 1e-14
    back = S.inverse(uh)
    assert tuple(back.shape) == (3, 3 * n // 2, 3 * n // 2, 3 * n // 2)
    assert torch.max(torch.abs(back - u)).item() <= 1e-14


def test_padded_ensemble_matches_single_samples(ns):
    sizes = [32, 16, 32]
    fields = [inputs.shear_layer(3 * n // 2, seed=30 + i)[0] for i, n in enumerate(sizes)]
    dts = [inputs.cfl_dt(u) for u in fields]
    E = ns.Solver(sizes, dtype=torch.float64, pad=True)
    uhs = E.forward([torch.from_numpy(u).cuda() for u in fields])
    E.step(uhs, dts, 3)
    for i, n in enumerate(sizes):
        S = ns.Solver(n, dtype=torch.float64, pad=True)
        uh = S.forward(torch.from_numpy(fields[i]).cuda())
        S.step(uh, dts[i], 3)
        assert torch.equal(uh, uhs[i]), i


def test_padded_rejects_unsupported_mode_counts(ns):
    for n in (30, 7, 2048):
        with pytest.raises(ns.NSError):
            ns.Solver(n, pad=True)


@pytest.mark.parametrize("n,dtype,tol", [(128, torch.float32, 1e-5), (256, torch.float64, 1e-12),
                                         (512, torch.float32, 1e-5), (1024, torch.float32, 1e-5)])
def test_padded_variants_full_size(ns, orc, n, dtype, tol):
    """Every schedule variant of every pass at the padded grids (radix-3, 6
    and 12 plans), one at a time, on a sparse field with modes on the cutoff
    edges, against the triad sum."""
    K = n // 2 - 1
    modes, coefs = inputs.sparse_modes(n, seed=n + 33, count=12, kmax=K)
    kout = _support(modes, K)
    ref = orc.rhs_sparse(modes, coefs, kout, n, orc.Params(kcut=K))
    cd = torch.complex128 if dtype == torch.float64 else torch.complex64
    S = ns.Solver(n, dtype=dtype, graph=False, pad=True)
    uh = torch.zeros((3, n, n, n // 2 + 1), dtype=cd, device="cuda")
    sel = modes[:, 0] >= 0
    for c in range(3):
        uh[c, torch.as_tensor(modes[sel, 2] % n), torch.as_tensor(modes[sel, 1] % n),
           torch.as_tensor(modes[sel, 0])] = torch.as_tensor(coefs[sel, c]).to(cd).cuda()
    oz, oy, ox = (torch.as_tensor(kout[:, 2] % n), torch.as_tensor(kout[:, 1] % n), torch.as_tensor(kout[:, 0]))
    for p in range(5):
        for v in range(S.variant_count(n, p)):
            S.set_variant(n, p, v)
            print("padded n=%d pass %d variant %d" % (n, p, v), flush=True)
            F = S.rhs(uh)
            got = torch.stack([F[c, oz, oy, ox] for c in range(3)], dim=1).cpu().numpy().astype(np.complex128)
            del F
            assert rel(got, ref) <= tol, (p, v)
        S.set_variant(n, p, 0)
