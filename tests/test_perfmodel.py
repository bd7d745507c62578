"""The byte-counting model: the paper's lower-bound formulas reproduce its
Table 2, and the pass model counts the bytes of the pruned passes."""
import os

import pytest

from paper_2401_09843_amd import perfmodel as pm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_lower_bounds.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_reproduces_table2():
    g = golden()
    N, p, s = 512, 8, 4
    bD, bHD = 488.64e9, 19.24e9
    got = {
        "padding": pm.t_pad(N, p, s, bD),
        "unpadding": pm.t_unpad(N, p, s, bD),
        "transpose_u": 3 * pm.t_transpose(N, p, s, bD, bHD, 9e9),
        "transpose_B": 6 * pm.t_transpose(N, p, s, bD, bHD, 9e9),
        "transpose_u_alltoall": 3 * pm.t_transpose(N, p, s, bD, bHD, 4e9),
        "transpose_B_alltoall": 6 * pm.t_transpose(N, p, s, bD, bHD, 4e9),
    }
    for k, v in g.items():
        assert got[k] * 1e3 == pytest.approx(v, abs=6e-4), k


def test_pass_model_hand_count():
    # N = 8: K = 2, M = 5, Mx = 3
    c = pm.pass_cw(8, 2)
    assert c["I1_inv_z"] == 3 * 25 * 3 + 3 * 8 * 5 * 3
    assert c["I2_inv_y"] == 3 * 8 * 5 * 3 + 3 * 64 * 3
    assert c["X_c2r_prod_r2c"] == 9 * 64 * 3
    assert c["F2_fwd_y"] == 6 * 64 * 3 + 6 * 8 * 5 * 3
    assert c["F3_fwd_z_epilogue"] == 6 * 8 * 5 * 3 + 9 * 75
    assert pm.pass_cw(8, 1)["F3_fwd_z_epilogue"] == 6 * 8 * 5 * 3 + 6 * 75


def test_step_bytes_1024():
    b = pm.step_bytes(1024, 4)
    assert 299e9 < b < 301e9  # about 34.97 N^3 complex words
    assert b / (8 * 1024 ** 3) == pytest.approx(34.97, abs=0.01)


def test_fused_model():
    # N = 8: K = 2, M = 5, Mx = 3, state 3 * 75, I1 output 3 * 120 complex words.
    # Fused, F3 also writes the next stage's I1 output; a step drops the
    # three I1 launches (three reads of the state saved), and one I1 per
    # call starts the chain.
    n, cw = 8, 8
    assert pm.pass_cw(n, 2, True)["F3_fwd_z_epilogue"] == pm.pass_cw(n, 2)["F3_fwd_z_epilogue"] + 3 * 120
    base = pm.step_bytes(n, 4)
    assert pm.step_bytes(n, 4, fused=True, steps_per_call=10 ** 12) == pytest.approx(base - cw * 3 * 225)
    assert pm.step_bytes(n, 4, fused=True, steps_per_call=1) == pytest.approx(base - cw * 3 * 225 + cw * 585)
    bpl = pm.pass_bytes_per_launch(n, 4, fused=True)
    assert bpl["F3_fwd_z_epilogue"] == pytest.approx(pm.pass_bytes_per_launch(n, 4)["F3_fwd_z_epilogue"] + cw * 360)


def test_adjoint_step_bytes_against_a_forward_step():
    """An adjoint step (three VJPs from a tape) moves about 1.3 times the
    bytes of a forward step: each VJP inverse-transforms eight fields (five
    strain components and three velocity components) where a right-hand
    side inverse-transforms three and forward-transforms six."""
    from paper_2401_09843_amd import perfmodel

    for n in (32, 128, 1024):
        r = perfmodel.adjoint_step_bytes(n, 8) / perfmodel.step_bytes(n, 8)
        assert 1.2 < r < 1.45, (n, r)
        K, M, Mx = perfmodel.dims(n)
        v = perfmodel.vjp_cw(n, 3)
        assert v["I1_inv_z"] == 6 * M * M * Mx + 8 * n * M * Mx  # lam and u in, eight fields out
        assert v["X_adj"] == 11 * n * n * Mx
