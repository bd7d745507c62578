"""Thin ctypes binding of libns.so (include/ns.h).

Only argument marshalling happens here: tensors are passed as device
pointers and every step of the computation runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: if the library or a GPU is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

from . import revolve

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libns.so")

NS_OK, NS_ERR_ARG, NS_ERR_UNSUPPORTED, NS_ERR_OOM, NS_ERR_HIP, NS_ERR_STATE, NS_ERR_NONFINITE = range(7)
NS_F32, NS_F64 = 0, 1
NS_USE_GRAPH, NS_CHECK_FINITE, NS_NO_TUNE, NS_NO_FUSE, NS_FUSE, NS_PAD = 1, 2, 4, 8, 16, 32
NS_GRAPH_CHAIN, NS_GRAPH_BRANCHES = 64, 128

# every symbol the header declares
EXPORTS = ("ns_init", "ns_destroy", "ns_last_error", "ns_workspace_bytes", "ns_supported_sizes", "ns_forward",
           "ns_inverse", "ns_project", "ns_rhs", "ns_step", "ns_tape_bytes", "ns_tape_step_bytes", "ns_step_taped",
           "ns_adjoint_step", "ns_adjoint_steps",
           "ns_energy_spectrum", "ns_enstrophy_spectrum", "ns_moments", "ns_structure_functions",
           "ns_wasserstein1", "ns_sync", "ns_profile", "ns_profile_read",
           "ns_variant_count", "ns_set_variant", "ns_tune_report", "ns_rhs_noalloc")
NS_NPASS = 5
PASS_NAMES = ("I1_inv_z", "I2_inv_y", "X_c2r_prod_r2c", "F2_fwd_y", "F3_fwd_z_epilogue")


class NSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("ns status %d: %s" % (status, msg))
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("nsamples", ctypes.c_int32), ("n", ctypes.POINTER(ctypes.c_int32)),
                ("eps", ctypes.c_double), ("s", ctypes.c_double), ("m_cut", ctypes.c_double),
                ("q_kind", ctypes.c_int32), ("theta", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("tune_cache", ctypes.c_char_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libns.so (built in-tree by paper_2401_09843_amd/_build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libns.so is not built (%s); run python -m paper_2401_09843_amd._build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I32, D, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        PP = ctypes.POINTER(ctypes.c_void_p)
        PD = ctypes.POINTER(ctypes.c_double)
        sig = {
            "ns_init": [ctypes.POINTER(_Params), P, ctypes.POINTER(P)],
            "ns_destroy": [P],
            "ns_workspace_bytes": [P, ctypes.POINTER(S)],
            "ns_supported_sizes": [ctypes.POINTER(I32), I32, ctypes.POINTER(I32)],
            "ns_forward": [P, PP, PP],
            "ns_inverse": [P, PP, PP],
            "ns_project": [P, PP],
            "ns_rhs": [P, PP, PP],
            "ns_step": [P, PP, PD, I32],
            "ns_tape_bytes": [P, I32, ctypes.POINTER(S)],
            "ns_tape_step_bytes": [P, I32, ctypes.POINTER(S)],
            "ns_step_taped": [P, PP, PD, I32, PP],
            "ns_adjoint_step": [P, PP, PP, PD, PP],
            "ns_adjoint_steps": [P, PP, I32, PD, PP],
            "ns_energy_spectrum": [P, PP, P, I32],
            "ns_enstrophy_spectrum": [P, PP, P, I32],
            "ns_moments": [P, PP, I32, P, P],
            "ns_wasserstein1": [P, P, I32, P, I32, I32, P, P],
            "ns_structure_functions": [P, PP, I32, D, P],
            "ns_sync": [P],
            "ns_profile": [P, I32],
            "ns_profile_read": [P, PD, ctypes.POINTER(ctypes.c_int64)],
            "ns_variant_count": [P, I32, I32, ctypes.POINTER(I32)],
            "ns_set_variant": [P, I32, I32, I32],
            "ns_tune_report": [P, ctypes.c_char_p, S, ctypes.POINTER(S)],
            "ns_rhs_noalloc": [ctypes.POINTER(_Params), P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.ns_last_error.argtypes = [P]
        L.ns_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def supported_sizes() -> list:
    L = lib()
    buf = (ctypes.c_int32 * 64)()
    cnt = ctypes.c_int32()
    L.ns_supported_sizes(buf, 64, ctypes.byref(cnt))
    return list(buf[: cnt.value])


def _ptrs(ts: Sequence[torch.Tensor]):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


class Solver:
    """A context for one sample (n = int) or an ensemble (n = list of ints).

    Spectra are complex tensors [3, N, N, N//2+1] (torch.fft.rfftn layout,
    norm="forward"); physical fields are real tensors [3, N, N, N].  Methods
    taking `uhat` accept a tensor (single sample) or a list of tensors.
    fuse: True ends every SSP-RK3 stage in the fused forward z + inverse z
    pass, False runs plain five-pass stages, None lets the autotuner time
    both per grid size (fused if tune is False).
    pad: Algorithm 2 in its padded form.  n is then the number of modes per
    axis of the state (spectra [3, n, n, n//2+1], modes |k_i| <= n/2 - 1) and
    the passes and physical fields use the grid of 3n/2 points.
    graph_form: with several grid sizes, "chain" runs the size groups of the
    captured step one after another, "branches" as concurrent graph
    branches; None lets the autotuner time both (chain if tune is False)."""

    def __init__(self, n, dtype=torch.float32, eps=-1.0, s=1.5, m_cut=-1.0, q_kind=0, theta=1.0,
                 graph=True, check_finite=False, tune=False, tune_cache=None, stream=None, device=None,
                 fuse=None, pad=False, graph_form=None):
        self.sizes = [int(n)] if isinstance(n, int) else [int(v) for v in n]
        self.pad = bool(pad)
        self.grids = [3 * v // 2 if self.pad else v for v in self.sizes]
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.cdtype = torch.complex64 if dtype == torch.float32 else torch.complex128
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._L = lib()
        nn = (ctypes.c_int32 * len(self.sizes))(*self.sizes)
        flags = ((NS_USE_GRAPH if graph else 0) | (NS_CHECK_FINITE if check_finite else 0)
                 | (0 if tune else NS_NO_TUNE) | {None: 0, True: NS_FUSE, False: NS_NO_FUSE}[fuse]
                 | (NS_PAD if self.pad else 0)
                 | {None: 0, "chain": NS_GRAPH_CHAIN, "branches": NS_GRAPH_BRANCHES}[graph_form])
        self._cache = tune_cache.encode() if tune_cache else None
        self._prm = _Params(NS_F32 if dtype == torch.float32 else NS_F64, len(self.sizes), nn, eps, s, m_cut,
                            q_kind, theta, flags, self._cache)
        self._nn = nn
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self._L.ns_init(ctypes.byref(self._prm), ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(ctx))
        if st != NS_OK:
            raise NSError(st, self._L.ns_last_error(None).decode())
        self._ctx = ctx

    # ------------------------------------------------------------ helpers
    def _check(self, st):
        if st != NS_OK:
            raise NSError(st, self._L.ns_last_error(self._ctx).decode())

    def _list(self, x):
        xs = [x] if isinstance(x, torch.Tensor) else list(x)
        if len(xs) != len(self.sizes):
            raise ValueError("expected %d tensors, got %d" % (len(self.sizes), len(xs)))
        return xs

    def _spec(self, xs):
        for t, n in zip(xs, self.sizes):
            if t.dtype != self.cdtype or t.device != self.device or not t.is_contiguous() \
                    or tuple(t.shape) != (3, n, n, n // 2 + 1):
                raise ValueError("spectrum must be a contiguous %s tensor [3,%d,%d,%d] on %s"
                                 % (self.cdtype, n, n, n // 2 + 1, self.device))
        return xs

    def _phys(self, xs):
        for t, n in zip(xs, self.grids):
            if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != (3, n, n, n):
                raise ValueError("field must be a contiguous %s tensor [3,%d,%d,%d] on %s"
                                 % (self.dtype, n, n, n, self.device))
        return xs

    def _ret(self, x, outs):
        return outs[0] if isinstance(x, torch.Tensor) else outs

    def empty_spectrum(self):
        return [torch.empty((3, n, n, n // 2 + 1), dtype=self.cdtype, device=self.device) for n in self.sizes]

    # ------------------------------------------------------------ API
    def forward(self, u):
        xs = self._phys(self._list(u))
        outs = self.empty_spectrum()
        self._check(self._L.ns_forward(self._ctx, _ptrs(xs), _ptrs(outs)))
        return self._ret(u, outs)

    def inverse(self, uhat):
        xs = self._spec(self._list(uhat))
        outs = [torch.empty((3, n, n, n), dtype=self.dtype, device=self.device) for n in self.grids]
        self._check(self._L.ns_inverse(self._ctx, _ptrs(xs), _ptrs(outs)))
        return self._ret(uhat, outs)

    def project(self, uhat):
        xs = self._spec(self._list(uhat))
        self._check(self._L.ns_project(self._ctx, _ptrs(xs)))
        return uhat

    def rhs(self, uhat):
        xs = self._spec(self._list(uhat))
        outs = self.empty_spectrum()
        self._check(self._L.ns_rhs(self._ctx, _ptrs(xs), _ptrs(outs)))
        return self._ret(uhat, outs)

    def step(self, uhat, dt, nsteps: int = 1):
        xs = self._spec(self._list(uhat))
        dts = [float(dt)] * len(xs) if not isinstance(dt, (list, tuple)) else [float(v) for v in dt]
        arr = (ctypes.c_double * len(dts))(*dts)
        self._check(self._L.ns_step(self._ctx, _ptrs(xs), arr, int(nsteps)))
        return uhat

    def tape_step_bytes(self, n: int) -> int:
        """Bytes of one step of the tape of a sample of size n (three compact
        stage states), as the library lays it out."""
        b = ctypes.c_size_t()
        self._check(self._L.ns_tape_step_bytes(self._ctx, int(n), ctypes.byref(b)))
        return int(b.value)

    def new_tape(self, nsteps: int):
        return [torch.empty(max(1, nsteps * self.tape_step_bytes(n)), dtype=torch.uint8, device=self.device)
                for n in self.sizes]

    def step_taped(self, uhat, dt, nsteps: int, tape):
        xs = self._spec(self._list(uhat))
        dts = [float(dt)] * len(xs) if not isinstance(dt, (list, tuple)) else [float(v) for v in dt]
        arr = (ctypes.c_double * len(dts))(*dts)
        tps = self._list(tape)
        for t, n in zip(tps, self.sizes):
            if t.device != self.device or t.numel() < nsteps * self.tape_step_bytes(n):
                raise ValueError("tape too small")
        self._check(self._L.ns_step_taped(self._ctx, _ptrs(xs), arr, int(nsteps), _ptrs(tps)))
        return uhat

    def adjoint_step(self, lam, dt, uhat_n=None, tape=None, step: int = 0):
        """lam: dJ/du^{n+1} -> dJ/du^n in place.  Stage states from step
        `step` of `tape` (from step_taped) or recomputed from uhat_n."""
        ls = self._spec(self._list(lam))
        dts = [float(dt)] * len(ls) if not isinstance(dt, (list, tuple)) else [float(v) for v in dt]
        arr = (ctypes.c_double * len(dts))(*dts)
        if tape is not None:
            tps = self._list(tape)
            tp = (ctypes.c_void_p * len(tps))()
            for i, (t, n) in enumerate(zip(tps, self.sizes)):
                off = step * self.tape_step_bytes(n)
                if off + self.tape_step_bytes(n) > t.numel():
                    raise ValueError("tape step out of range")
                tp[i] = t.data_ptr() + off
            self._check(self._L.ns_adjoint_step(self._ctx, None, tp, arr, _ptrs(ls)))
        else:
            us = self._spec(self._list(uhat_n))
            self._check(self._L.ns_adjoint_step(self._ctx, _ptrs(us), None, arr, _ptrs(ls)))
        return lam

    def adjoint_steps(self, lam, dt, tape, nsteps: int):
        """nsteps adjoint steps backward through a tape from step_taped."""
        ls = self._spec(self._list(lam))
        dts = [float(dt)] * len(ls) if not isinstance(dt, (list, tuple)) else [float(v) for v in dt]
        arr = (ctypes.c_double * len(dts))(*dts)
        tps = self._list(tape)
        for t, n in zip(tps, self.sizes):
            if t.device != self.device or t.numel() < nsteps * self.tape_step_bytes(n):
                raise ValueError("tape too small")
        self._check(self._L.ns_adjoint_steps(self._ctx, _ptrs(tps), int(nsteps), arr, _ptrs(ls)))
        return lam

    def enstrophy_spectrum(self, uhat, kbins: int):
        xs = self._spec(self._list(uhat))
        Z = torch.zeros((len(xs), kbins), dtype=torch.float64, device=self.device)
        self._check(self._L.ns_enstrophy_spectrum(self._ctx, _ptrs(xs), ctypes.c_void_p(Z.data_ptr()), int(kbins)))
        return Z

    def moments(self, uhat, n: int):
        """Pointwise mean and variance (1/B) of the physical velocity over
        the samples of size n: two float64 tensors [3, N, N, N]."""
        xs = self._spec(self._list(uhat))
        if n not in self.sizes:
            raise ValueError("no samples of size %d" % n)
        N = self.grids[self.sizes.index(n)]
        mean = torch.empty((3, N, N, N), dtype=torch.float64, device=self.device)
        var = torch.empty_like(mean)
        self._check(self._L.ns_moments(self._ctx, _ptrs(xs), int(n), ctypes.c_void_p(mean.data_ptr()),
                                       ctypes.c_void_p(var.data_ptr())))
        return mean, var

    def structure_functions(self, uhat, lmax: int, p: float):
        """Longitudinal structure functions of order p for shifts 1..lmax
        grid points: float64 [nsamples, lmax]."""
        xs = self._spec(self._list(uhat))
        S = torch.empty((len(xs), lmax), dtype=torch.float64, device=self.device)
        self._check(self._L.ns_structure_functions(self._ctx, _ptrs(xs), int(lmax), float(p),
                                                   ctypes.c_void_p(S.data_ptr())))
        return S

    def wasserstein1(self, a: torch.Tensor, b: torch.Tensor):
        """Pointwise W1 between the 1-point marginals (component by
        component) of two ensembles of physical fields a [na, 3, n, n, n] and
        b [nb, 3, n, n, n]: returns (w [3, n, n, n], mean over points [3]),
        float64."""
        for t in (a, b):
            if t.dim() != 5 or t.shape[1] != 3 or t.dtype != self.dtype or t.device != self.device \
                    or not t.is_contiguous() or not (t.shape[2] == t.shape[3] == t.shape[4]):
                raise ValueError("ensembles must be contiguous %s tensors [m, 3, n, n, n] on %s"
                                 % (self.dtype, self.device))
        if a.shape[2:] != b.shape[2:]:
            raise ValueError("the two ensembles must share the grid")
        n = a.shape[-1]
        w = torch.empty(a.shape[1:], dtype=torch.float64, device=self.device)
        mean = torch.empty(3, dtype=torch.float64, device=self.device)
        self._check(self._L.ns_wasserstein1(self._ctx, ctypes.c_void_p(a.data_ptr()), int(a.shape[0]),
                                            ctypes.c_void_p(b.data_ptr()), int(b.shape[0]), int(n),
                                            ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(mean.data_ptr())))
        return w, mean

    def spectrum(self, uhat, kbins: int):
        xs = self._spec(self._list(uhat))
        E = torch.zeros((len(xs), kbins), dtype=torch.float64, device=self.device)
        self._check(self._L.ns_energy_spectrum(self._ctx, _ptrs(xs), ctypes.c_void_p(E.data_ptr()), int(kbins)))
        return E

    def profile(self, enable: bool = True):
        self._check(self._L.ns_profile(self._ctx, 1 if enable else 0))

    def profile_read(self):
        """{pass name: (total ms, launches)} since the last read."""
        ms = (ctypes.c_double * NS_NPASS)()
        cnt = (ctypes.c_int64 * NS_NPASS)()
        self._check(self._L.ns_profile_read(self._ctx, ms, cnt))
        return {PASS_NAMES[p]: (ms[p], cnt[p]) for p in range(NS_NPASS)}

    def variant_count(self, n: int, p: int) -> int:
        c = ctypes.c_int32()
        self._check(self._L.ns_variant_count(self._ctx, int(n), int(p), ctypes.byref(c)))
        return c.value

    def set_variant(self, n: int, p: int, v: int):
        self._check(self._L.ns_set_variant(self._ctx, int(n), int(p), int(v)))

    def tune_report(self):
        import json
        need = ctypes.c_size_t()
        self._check(self._L.ns_tune_report(self._ctx, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        self._check(self._L.ns_tune_report(self._ctx, buf, need.value, ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def workspace_bytes(self) -> int:
        v = ctypes.c_size_t()
        self._check(self._L.ns_workspace_bytes(self._ctx, ctypes.byref(v)))
        return v.value

    def sync(self):
        self._check(self._L.ns_sync(self._ctx))

    def close(self):
        if getattr(self, "_ctx", None):
            self._L.ns_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 64 << 20


def rhs_noalloc(uhat: torch.Tensor, out: torch.Tensor = None, eps=-1.0, s=1.5, m_cut=-1.0, q_kind=0, theta=1.0,
                pad=False, stream=None) -> torch.Tensor:
    """ns_rhs_noalloc: the right-hand side of one spectrum uhat [3, n, n, n//2+1]
    (complex64 or complex128, contiguous, on the current device) without a
    context; the library allocates nothing (its workspaces are a static
    device array of NOALLOC_SCRATCH_BYTES per GPU).  Equals ns_rhs of a
    Solver(n, tune=False, pad=pad) with the same parameters, bit for bit.
    out: preallocated output of uhat's shape and dtype (else one is made
    here, by torch)."""
    if uhat.dtype not in (torch.complex64, torch.complex128) or not uhat.is_contiguous() or uhat.dim() != 4 \
            or uhat.shape[0] != 3 or not (uhat.shape[1] == uhat.shape[2] == 2 * (uhat.shape[3] - 1)):
        raise ValueError("uhat must be a contiguous complex tensor [3, n, n, n//2+1]")
    if out is None:
        out = torch.empty_like(uhat)
    elif out.shape != uhat.shape or out.dtype != uhat.dtype or not out.is_contiguous() or out.device != uhat.device:
        raise ValueError("out must be a contiguous tensor like uhat")
    L = lib()
    n = int(uhat.shape[1])
    nn = (ctypes.c_int32 * 1)(n)
    prm = _Params(NS_F32 if uhat.dtype == torch.complex64 else NS_F64, 1, nn, eps, s, m_cut, q_kind, theta,
                  NS_PAD if pad else 0, None)
    st = stream if stream is not None else torch.cuda.current_stream(uhat.device)
    with torch.cuda.device(uhat.device):
        code = L.ns_rhs_noalloc(ctypes.byref(prm), ctypes.c_void_p(uhat.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(st.cuda_stream))
    if code != NS_OK:
        raise NSError(code, L.ns_last_error(None).decode())
    return out


class _Rollout(torch.autograd.Function):
    """u0 (physical) -> u(T) (physical) after nsteps SSP-RK3 steps, with the
    discrete adjoint in backward.  The trajectory is cut into segments of
    `ckpt_every` steps, the unit of reversal: a segment is reversed by
    re-running it from its start state with its stage tape recorded
    (ns_step_taped), then stepping the adjoint back through the tape
    (ns_adjoint_steps).  If the stage tape of the whole trajectory fits the
    memory budget it is recorded during the forward pass and the backward
    only runs the adjoint.  Otherwise the segment start states are kept by
    the binomial (revolve) schedule for `snapshots` checkpoint slots: the
    forward pass runs the schedule up to its first reversal (the last
    segment, taped on the way to the output) and the backward runs the rest.
    With a slot for every segment start (the default) this is the uniform
    scheme: every segment but the last is re-run once.

    Gradient algebra: u(T) = F^-1[T u-hat(T)] and u-hat(0) = T P F[u0], with
    F normalised by N^-3.  In the inner product Re sum_k conj(a_k) b_k the
    adjoint of the first map is N^3 T F and of the second N^-3 F^-1 P T, so
    with lambda(T) = T P F[g] (the solver's ns_forward) and the gradient
    F^-1[P T lambda(0)] (ns_project then ns_inverse) the two factors cancel.
    The projection added at the seed only removes a component that the
    final projection removes anyway (the divergent part of lambda evolves
    on its own)."""

    @staticmethod
    def forward(ctx, u0, solver, dt, nsteps, ckpt_every, tape_budget, snapshots, stats):
        uh = solver.forward(u0.detach().contiguous())
        L = ckpt_every
        nseg = (nsteps + L - 1) // L
        lens = [min(L, nsteps - i * L) for i in range(nseg)]
        total = nsteps * solver.tape_step_bytes(solver.sizes[0])
        ctx.solver, ctx.dt, ctx.lens, ctx.stats = solver, dt, lens, stats
        taped = nsteps
        if total <= tape_budget:
            # one tape, written segment by segment: every mode makes the same
            # calls per segment (a call may start its stages differently in the
            # fused form), so all modes follow the same trajectory bit for bit
            tape = solver.new_tape(nsteps)[0]
            per = solver.tape_step_bytes(solver.sizes[0])
            for i, n in enumerate(lens):
                solver.step_taped(uh, dt, n, tape[i * L * per:])
            ctx.tape, ctx.rest = tape, None
            if stats is not None:
                stats.update({"mode": "whole tape", "segments": nseg, "snapshots": 0})
            return solver.inverse(uh)
        c = nseg - 1 if snapshots is None else max(0, min(int(snapshots), nseg - 1))
        acts = revolve.schedule(nseg, c)
        ctx.state0 = uh.clone()
        snaps = {}
        advanced = 0
        k = 0
        while acts[k][0] != revolve.REVERSE:
            a = acts[k]
            if a[0] == revolve.ADVANCE:
                for n in lens[a[1]:a[2]]:  # one call per segment, as everywhere
                    solver.step(uh, dt, n)
                    advanced += n
            elif a[0] == revolve.TAKESHOT:
                snaps[a[1]] = uh.clone()
            else:
                raise RuntimeError("unexpected action %r before the first reversal" % (a,))
            k += 1
        # the first reversal is that of the last segment, from the current
        # state: taped on the way to the output
        assert acts[k] == (revolve.REVERSE, nseg - 1)
        tape = solver.new_tape(lens[-1])[0]
        solver.step_taped(uh, dt, lens[-1], tape)
        ctx.tape, ctx.rest, ctx.snaps = tape, acts[k + 1:], snaps
        ctx.counts = [advanced + lens[-1], lens[-1]]
        if stats is not None:
            stats.update({"mode": "revolve", "segments": nseg, "snapshots": c,
                          "schedule_forward_segments": revolve.forward_steps(acts)})
        return solver.inverse(uh)

    @staticmethod
    def backward(ctx, g):
        S, dt, lens = ctx.solver, ctx.dt, ctx.lens
        lam = S.forward(g.detach().contiguous().to(S.dtype))
        if ctx.rest is None:
            S.adjoint_steps(lam, dt, ctx.tape, sum(lens))
            ctx.tape = None
            if ctx.stats is not None:
                ctx.stats.update({"forward_steps": sum(lens), "taped_steps": sum(lens)})
        else:
            S.adjoint_steps(lam, dt, ctx.tape, lens[-1])
            ctx.tape = None
            fwd, taped = ctx.counts
            cur = None
            for a in ctx.rest:
                if a[0] == revolve.ADVANCE:
                    for n in lens[a[1]:a[2]]:
                        S.step(cur, dt, n)
                        fwd += n
                elif a[0] == revolve.TAKESHOT:
                    ctx.snaps[a[1]] = cur.clone()
                elif a[0] == revolve.RESTORE:
                    cur = (ctx.state0 if a[1] == 0 else ctx.snaps[a[1]]).clone()
                elif a[0] == revolve.FREE:
                    del ctx.snaps[a[1]]
                else:  # REVERSE: re-run segment a[1] taped, then the adjoint back through it
                    n = lens[a[1]]
                    tape = S.new_tape(n)[0]
                    S.step_taped(cur, dt, n, tape)
                    S.adjoint_steps(lam, dt, tape, n)
                    fwd += n
                    taped += n
                    del tape
                    cur = None
            ctx.snaps = None
            ctx.state0 = None
            if ctx.stats is not None:
                ctx.stats.update({"forward_steps": fwd, "taped_steps": taped})
        S.project(lam)
        return S.inverse(lam), None, None, None, None, None, None, None


def rollout(u0: torch.Tensor, solver: "Solver", dt: float, nsteps: int, ckpt_every: int = 20,
            tape_budget: int = None, snapshots: int = None, stats: dict = None) -> torch.Tensor:
    """Differentiable SSP-RK3 trajectory of a single-sample solver:
    physical u0 [3,N,N,N] -> physical u(T) after nsteps steps of size dt.
    tape_budget: bytes of device memory the full stage tape may use to avoid
    recomputation (default: a quarter of the free device memory; 0 forces
    checkpointing with recomputation in segments of ckpt_every steps).
    snapshots: checkpoint slots for segment start states when checkpointing
    (None: one per segment, i.e. uniform checkpoints every ckpt_every steps;
    fewer slots follow the binomial revolve schedule and re-run more).
    stats: if a dict, receives the mode and the number of forward steps run
    (taped re-runs included)."""
    if len(solver.sizes) != 1:
        raise ValueError("rollout needs a single-sample solver")
    if tape_budget is None:
        free, _ = torch.cuda.mem_get_info(solver.device)
        tape_budget = free // 4
    return _Rollout.apply(u0, solver, float(dt), int(nsteps), int(ckpt_every), int(tape_budget),
                          snapshots, stats)
