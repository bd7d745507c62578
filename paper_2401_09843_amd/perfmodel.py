"""Algorithmic byte counts of the passes and the paper's kernel lower bounds.

Counting rule (Sec. 5.1): every element a pass needs is read once from HBM
and every element it produces is written once; zeros are never stored.
Sizes per axis: K = floor((N-1)/3), M = 2K+1 retained wavenumbers on a full
axis, Mx = K+1 on the half (R2C) axis.  One complex word (cw) is 2 reals.
"""
from __future__ import annotations

PASSES = ("I1_inv_z", "I2_inv_y", "X_c2r_prod_r2c", "F2_fwd_y", "F3_fwd_z_epilogue")


def dims(n: int):
    K = (n - 1) // 3
    return K, 2 * K + 1, K + 1


def pass_cw(n: int, stage: int = 2, fused: bool = False) -> dict:
    """Complex words moved per pass for one right-hand side of one sample.
    stage 1 of SSP-RK3 reads one state and writes one; stages 2 and 3 read
    two states (u^n and the stage state) and write one.  fused: F3 also
    writes the inverse z transform of the new state (the next stage's I1
    output), so that the next stage skips I1 and its read of the state."""
    K, M, Mx = dims(n)
    st = M * M * Mx
    state_io = 6 * st if stage == 1 else 9 * st
    return {
        "I1_inv_z": 3 * st + 3 * n * M * Mx,
        "I2_inv_y": 3 * n * M * Mx + 3 * n * n * Mx,
        "X_c2r_prod_r2c": 3 * n * n * Mx + 6 * n * n * Mx,
        "F2_fwd_y": 6 * n * n * Mx + 6 * n * M * Mx,
        "F3_fwd_z_epilogue": 6 * n * M * Mx + state_io + (3 * n * M * Mx if fused else 0),
    }


def pass_bytes_per_launch(n: int, real_bytes: int, batch: int = 1, fused: bool = False) -> dict:
    """Algorithmic bytes of one launch of each pass, averaged over the three
    RK3 stages (only F3 differs between stages)."""
    cw = 2 * real_bytes
    s1, s2 = pass_cw(n, 1, fused), pass_cw(n, 2, fused)
    out = {}
    for p in PASSES:
        out[p] = batch * cw * (s1[p] + 2 * s2[p]) / 3.0
    return out


def step_bytes(n: int, real_bytes: int, fused: bool = False, steps_per_call: int = 1) -> float:
    """Algorithmic HBM bytes of one SSP-RK3 step of one sample.  Fused, the
    three stages run I2, X, F2 and the fused F3, and one I1 per call of
    steps_per_call steps starts the chain."""
    cw = 2 * real_bytes
    s1, s2 = pass_cw(n, 1, fused), pass_cw(n, 2, fused)
    if not fused:
        return cw * (sum(s1.values()) + 2 * sum(s2.values()))
    per = sum(s1.values()) + 2 * sum(s2.values()) - 3 * s1["I1_inv_z"]
    return cw * (per + s1["I1_inv_z"] / steps_per_call)


def vjp_cw(n: int, stage: int) -> dict:
    """Complex words moved by one vector-Jacobian product of the right-hand
    side fused with adjoint RK3 stage `stage` (1: lambda_2, 2: lambda_1,
    3: lambda_n), one sample: a z pass that reads lam and u (three compact
    components each), forms the five stored components of the trace-free
    strain of P lam in registers and writes the inverse z transforms of
    those five and of u, the inverse y pass of the eight, the x pass forming
    2 S u, forward y and z passes of its three components, and the stage
    epilogue, which reads lam and the earlier adjoint stages with nonzero
    coefficients (two arrays in stages 1 and 2, three in stage 3) and
    writes one."""
    K, M, Mx = dims(n)
    st = M * M * Mx
    reads = 3 if stage == 3 else 2
    return {
        "I1_inv_z": 6 * st + 8 * n * M * Mx,
        "I2_inv_y": 8 * n * M * Mx + 8 * n * n * Mx,
        "X_adj": 8 * n * n * Mx + 3 * n * n * Mx,
        "F2_fwd_y": 3 * n * n * Mx + 3 * n * M * Mx,
        "F3_adj": 3 * n * M * Mx + 3 * reads * st + 3 * st,
    }


def adjoint_step_bytes(n: int, real_bytes: int) -> float:
    """Algorithmic HBM bytes of one adjoint SSP-RK3 step (three VJPs) of one
    sample, reading its stage states from a tape."""
    return 2 * real_bytes * sum(sum(vjp_cw(n, s).values()) for s in (1, 2, 3))


# ---- the paper's lower bounds (Sec. 5.1, eqs. (5.1)-(5.3)), N grid, p ranks,
# s bytes per scalar, bandwidths in bytes/s
def t_pad(N, p, s, beta):
    return 213.0 / 16.0 * N ** 3 / p * 2 * s / beta


def t_unpad(N, p, s, beta):
    return 78.0 / 4.0 * N ** 3 / p * 2 * s / beta


def t_transpose(N, p, s, beta_d, beta_hd, beta_mpi):
    return (4.5 * N ** 3 / p ** 2 * 2 * s / beta_d + 2.25 * N ** 3 / p ** 2 * 2 * s / beta_hd
            + 1.125 * N ** 3 / p * 2 * s / beta_mpi)
