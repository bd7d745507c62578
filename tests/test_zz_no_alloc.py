"""The allocation-free right-hand side (ns_rhs_noalloc) against the context
entry point ns_rhs with the same built-in schedules, through the C ABI.

Two calls in a row per case, the second on a smaller grid, so the second
call runs on workspaces and tables that the first one left in the static
array.  The bar is the one of every right-hand-side parity test (1e-12
relative L2 in FP64, 1e-5 in FP32); the outputs are also expected to be
bitwise equal, since both run the same kernels on the same tables."""
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


def spectrum(n, seed, cdtype):
    uh = inputs.half_spectrum(inputs.random_field(n, seed=seed))
    return torch.from_numpy(uh).to("cuda", cdtype).contiguous()


def rel(a, b):
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return float(torch.linalg.vector_norm(a - b).item() / torch.linalg.vector_norm(b).item())


@pytest.mark.parametrize("dtype,sizes,pad,tol", [
    (torch.float64, (64, 32), False, 1e-12),
    (torch.float32, (96, 48), False, 1e-5),
    (torch.float32, (64, 32), True, 1e-5),  # padded form: grids 96 and 48
    (torch.float64, (80, 24), False, 1e-12),
])
def test_rhs_noalloc_matches_rhs(ns, dtype, sizes, pad, tol):
    cd = torch.complex64 if dtype == torch.float32 else torch.complex128
    for i, n in enumerate(sizes):
        print("rhs_noalloc %s n=%d pad=%s (call %d)" % (dtype, n, pad, i + 1), flush=True)
        uh = spectrum(n, seed=300 + n, cdtype=cd)
        out = torch.full_like(uh, float("nan"))
        ns.rhs_noalloc(uh, out=out, pad=pad)
        S = ns.Solver(n, dtype=dtype, tune=False, pad=pad)
        ref = S.rhs(uh)
        torch.cuda.synchronize()
        S.close()
        err = rel(out, ref)
        print("  rel L2 vs ns_rhs %.3e, bitwise equal %s" % (err, bool(torch.equal(out, ref))), flush=True)
        assert err <= tol
        assert torch.equal(out, ref)


def test_rhs_noalloc_against_the_oracle(ns, orc):
    n = 32
    uh = spectrum(n, seed=11, cdtype=torch.complex128)
    got = ns.rhs_noalloc(uh).cpu().numpy()
    ref = orc.rhs(uh.cpu().numpy(), n, orc.Params())
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_rhs_noalloc_rejects_sizes_beyond_the_array(ns):
    uh = torch.zeros((3, 128, 128, 65), dtype=torch.complex64, device="cuda")
    with pytest.raises(ns.NSError) as e:
        ns.rhs_noalloc(uh)
    assert e.value.status == ns.NS_ERR_ARG
    assert "scratch" in str(e.value)
