"""Every schedule variant the autotuner can pick computes the same
right-hand side: each pass's variants are forced one at a time (the other
passes at their default) and checked against the oracle, by the full
pseudo-spectral oracle at 64^3/128^3 and by the sparse Galerkin oracle at
256^3 (FP64) and 512^3/1024^3 (FP32)."""
import numpy as np
import pytest
import torch

from paper_2401_09843_amd import inputs

pytestmark = pytest.mark.gpu
NPASS = 5


@pytest.fixture(scope="module")
def ns():
    from paper_2401_09843_amd import ns as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def edge_errors(got, ref, n):
    """Per-mode maximum (relative to the largest mode) and the relative L2
    error on the cutoff faces and on the k_x = 0 plane, where an error in a
    variant's Hermitian handling or truncation could hide under a
    whole-array norm."""
    K = (n - 1) // 3
    kz = np.abs(np.fft.fftfreq(n, 1.0 / n))[:, None, None]
    ky = np.abs(np.fft.fftfreq(n, 1.0 / n))[None, :, None]
    kx = np.arange(n // 2 + 1)[None, None, :]
    faces = ((kz == K) | (ky == K) | (kx == K)) & (kz <= K) & (ky <= K) & (kx <= K)
    faces = np.broadcast_to(faces, got.shape[1:])
    plane0 = np.zeros(got.shape[1:], dtype=bool)
    plane0[:, :, 0] = True
    e_max = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    return e_max, rel(got[:, faces], ref[:, faces]), rel(got[:, plane0], ref[:, plane0])


def each_variant(S, n):
    for p in range(NPASS):
        for v in range(S.variant_count(n, p)):
            S.set_variant(n, p, v)
            yield p, v
        S.set_variant(n, p, 0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [64, 128])
def test_variants_small(ns, orc, n, dtype):
    uh = inputs.half_spectrum(inputs.random_field(n, seed=3000 + n))
    ref = orc.rhs(uh, n)
    cd = torch.complex128 if dtype == torch.float64 else torch.complex64
    S = ns.Solver(n, dtype=dtype, graph=False)
    x = torch.from_numpy(uh).to(cd).cuda()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for p, v in each_variant(S, n):
        print("n=%d %s pass %d variant %d" % (n, dtype, p, v), flush=True)
        got = S.rhs(x).cpu().numpy().astype(np.complex128)
        assert rel(got, ref) <= tol, (p, v)
        e_max, e_face, e_plane = edge_errors(got, ref, n)
        assert e_max <= tol and e_face <= 10 * tol and e_plane <= 10 * tol, (p, v, e_max, e_face, e_plane)


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
def test_variants_full_size(ns, orc, n, dtype, tol):
    modes, coefs = inputs.sparse_modes(n, seed=n + 11, count=16)
    kout = _support(modes, (n - 1) // 3)
    ref = orc.rhs_sparse(modes, coefs, kout, n, orc.Params())
    cd = torch.complex128 if dtype == torch.float64 else torch.complex64
    S = ns.Solver(n, dtype=dtype, graph=False)
    uh = torch.zeros((3, n, n, n // 2 + 1), dtype=cd, device="cuda")
    sel = modes[:, 0] >= 0
    for c in range(3):
        uh[c, torch.as_tensor(modes[sel, 2] % n), torch.as_tensor(modes[sel, 1] % n),
           torch.as_tensor(modes[sel, 0])] = torch.as_tensor(coefs[sel, c]).to(cd).cuda()
    oz, oy, ox = (torch.as_tensor(kout[:, 2] % n), torch.as_tensor(kout[:, 1] % n), torch.as_tensor(kout[:, 0]))
    for p, v in each_variant(S, n):
        print("n=%d pass %d variant %d" % (n, p, v), flush=True)
        F = S.rhs(uh)
        got = torch.stack([F[c, oz, oy, ox] for c in range(3)], dim=1).cpu().numpy().astype(np.complex128)
        total = float(torch.sum(torch.abs(F.to(torch.complex128)) ** 2).item())
        for c in range(3):
            F[c, oz, oy, ox] = 0
        off = float(torch.sum(torch.abs(F.to(torch.complex128)) ** 2).item())
        del F
        assert rel(got, ref) <= tol, (p, v)
        assert off <= 10 * tol ** 2 * total, (p, v)


def _dev(a, dtype):
    cd = torch.complex128 if dtype == torch.float64 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(cd).cuda()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [64, 128])
def test_fused_step_variants_small(ns, orc, n, dtype):
    """Stepping ends each stage in the fused form of F3 (it also writes the
    inverse z transform of the new state for the next stage, which then
    skips I1): two SSP-RK3 steps with each F3 variant, fused and plain,
    against the oracle."""
    u0, _, _ = inputs.shear_layer(n, seed=5)
    dt = inputs.cfl_dt(u0)
    ref0 = orc.initial_state(u0)
    ref = orc.ssprk3(ref0, n, dt, 2)
    tol = 1e-12 if dtype == torch.float64 else 5e-6
    for fuse in (True, False):
        S = ns.Solver(n, dtype=dtype, graph=False, fuse=fuse)
        for v in range(S.variant_count(n, 4)):
            print("n=%d %s fuse=%s F3 variant %d" % (n, dtype, fuse, v), flush=True)
            S.set_variant(n, 4, v)
            uh = _dev(ref0, dtype)
            S.step(uh, dt, 2)
            assert rel(uh.cpu().numpy().astype(np.complex128), ref) <= tol, (fuse, v)


@pytest.mark.parametrize("n,dtype", [(256, torch.float64), (512, torch.float32), (1024, torch.float32)])
def test_fused_step_variants_full_size(ns, n, dtype):
    """At full size, where the oracle has no whole step, each F3 variant's
    fused step against the plain five-pass step (whose passes the variant
    tests above pin to the oracle): two steps of the shear layer, with the
    graph replayed, to the precision's rounding."""
    u0, _, _ = inputs.shear_layer_torch(n, seed=0, device="cuda", dtype=dtype)
    dt = float(0.5 * (2 * np.pi / n) / u0.abs().sum(0).max().item())
    plain = ns.Solver(n, dtype=dtype, fuse=False)
    uh0 = plain.forward(u0)
    del u0
    ref = uh0.clone()
    plain.step(ref, dt, 2)
    del plain
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    S = ns.Solver(n, dtype=dtype)
    for v in range(S.variant_count(n, 4)):
        print("n=%d fused F3 variant %d" % (n, v), flush=True)
        S.set_variant(n, 4, v)
        uh = uh0.clone()
        S.step(uh, dt, 2)
        d = (torch.linalg.vector_norm(uh - ref) / torch.linalg.vector_norm(ref)).item()
        assert d <= tol, (v, d)
        del uh


def test_tuner_picks_a_listed_variant_and_caches(ns, tmp_path):
    n = 64
    path = str(tmp_path / "tune.jsonl")
    S = ns.Solver(n, dtype=torch.float32, tune=True, tune_cache=path)
    rep = S.tune_report()
    assert len(rep) == NPASS
    for r in rep:
        assert r["selected"] in r["timings_ms"]
    # the stage form: whole plain and fused stages were timed, the faster kept
    f3 = rep[-1]
    assert f3["stage_ms"]["plain"] > 0 and f3["stage_ms"]["fused"] > 0
    assert f3["fused"] == (f3["stage_ms"]["fused"] < f3["stage_ms"]["plain"])
    lines = open(path).read().strip().splitlines()
    assert len(lines) == NPASS + 1
    S2 = ns.Solver(n, dtype=torch.float32, tune=True, tune_cache=path)  # read back
    rep2 = S2.tune_report()
    assert [r["selected"] for r in rep2] == [r["selected"] for r in rep]
    assert rep2[-1]["fused"] == f3["fused"]
    # forced forms
    for fuse in (True, False):
        assert ns.Solver(n, dtype=torch.float32, tune=True, fuse=fuse).tune_report()[-1]["fused"] is fuse
