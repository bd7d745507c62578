"""Benchmark: SSP-RK3 steps of the spectral hyperviscosity solver on one MI355X.

Headline workload: the seeded perturbed shear layer at N = 1024^3, FP32,
s = 1.5, step multiplier at m_N = N/3, eps_N = 1e-3 (32/N)^2, dt from CFL 0.5;
W warm-up steps (graph replay), then K timed steps in one ns_step call, inputs
resident in HBM.  A stage runs the plain five passes or, in the fused form,
four (the forward z pass also writes the inverse z transform of the new
state); the autotuner picks the faster form (--fuse / --no-fuse force one).
The timed steps run with the pass profiler on: HIP events bracket every pass
launch on the library's stream (eager launches; --no-profile times graph
replays instead).

The default run prints one JSON line with:
  value / roofline      Mpts*RK-steps/s at 1024^3 FP32 and the HBM roofline of
                        its dominant pass (algorithmic bytes / its average
                        event-timed duration in the timed region)
  fp32_vs_fp64          relative L2 of the timed FP32 run's final spectrum
                        against an FP64 run of the same steps from the same
                        field (FP64 solver on the GPU)
  n512                  the same measurement at 512^3 FP32
  ensemble              96 samples (64 x 128^3 + 32 x 64^3, FP32, 200 steps):
                        batched samples/s against looping plain solvers, each
                        autotuned at one sample, plus the loop on the batched
                        schedules (bitwise equal to the batched result)
  cpu_baseline          the CPU oracle on a bounded sample of the same family

    python bench.py [--gpus 1] [--steps 20] [--warmup 2] [--n 1024] [--only-headline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
ENS_SIZES = [128] * 64 + [64] * 32
ENS_METRIC = "ensemble samples/s (96 samples: 64x128^3 + 32x64^3, 200 SSP-RK3 steps)"


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def mem_available_bytes() -> int:
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) * 1024
    except OSError:
        pass
    return 0


def cpu_baseline(n_step: int = 256, n_rhs: int = 512):
    """The oracle (FP64, its OpenMP threads) on a bounded sample of the
    shear-layer family: one SSP-RK3 step at n_step^3, and one right-hand side
    at n_rhs^3 when the host has the memory (an SSP-RK3 step is three
    right-hand sides plus O(N^3) combinations).  The 1024^3 figure is
    extrapolated by N^3 log N from the largest size measured."""
    import gc

    from oracle import oracle as orc
    from paper_2401_09843_amd import inputs

    u0, _, _ = inputs.shear_layer(n_step, seed=0)
    dt = inputs.cfl_dt(u0)
    uh = orc.initial_state(u0)
    del u0
    t0 = time.perf_counter()
    orc.ssprk3(uh, n_step, dt, 1)
    t_step = time.perf_counter() - t0
    del uh
    gc.collect()
    out = {"value": n_step ** 3 / t_step / 1e6, "unit": "Mpts*RK-steps/s", "cores": orc.num_threads(),
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "one SSP-RK3 step (3 RHS) of the seed-0 shear layer at %d^3, FP64, %.1f s" % (n_step, t_step)}
    base_n, base_t = n_step, t_step
    need = 24 * n_rhs ** 3 * 16  # the full complex arrays the oracle and its layout glue hold at once, with margin
    if mem_available_bytes() >= need:
        u0, _, _ = inputs.shear_layer(n_rhs, seed=0)
        uh = orc.initial_state(u0)
        del u0
        gc.collect()
        t0 = time.perf_counter()
        orc.rhs(uh, n_rhs)
        t_rhs = time.perf_counter() - t0
        del uh
        gc.collect()
        out["n%d_rhs_s" % n_rhs] = t_rhs
        out["n%d_step_s_from_rhs" % n_rhs] = 3 * t_rhs
        out["n%d_value_from_rhs" % n_rhs] = n_rhs ** 3 / (3 * t_rhs) / 1e6
        out["sample"] += "; one RHS at %d^3, %.1f s (a step is 3 RHS)" % (n_rhs, t_rhs)
        base_n, base_t = n_rhs, 3 * t_rhs
    else:
        out["n%d_rhs_s" % n_rhs] = None
        out["n%d_skipped" % n_rhs] = "host memory available %.0f GB < %.0f GB" % (mem_available_bytes() / 1e9, need / 1e9)
    t1024 = base_t * (1024 / base_n) ** 3 * math.log(1024) / math.log(base_n)
    out["extrapolated_1024"] = {"step_s": t1024, "value": 1024 ** 3 / t1024 / 1e6,
                                "label": "extrapolated by N^3 log N from %d^3 (not run)" % base_n}
    return out


def fuse_arg(args):
    """Stage form requested on the command line: None lets the autotuner
    choose."""
    if args.fuse and args.no_fuse:
        sys.exit("--fuse and --no-fuse exclude each other")
    return True if args.fuse else (False if args.no_fuse else None)


def kernel_source_hash(n: int = 1024) -> str:
    """SHA-256 of the device-code sources the pass kernels of grid size n are
    built from (the shared kernel headers and size_<n>.hip; not the host
    runtime); PMC traffic figures are valid only for the kernels they were
    measured on."""
    import glob
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2401_09843_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hpp")) + [os.path.join(csrc, "size_%d.hip" % n)]):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, n: int, variant: str, stage_form: str):
    """HBM bytes per launch of a pass from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None if there is none, the kernels changed since, or
    the figure belongs to another schedule variant or stage form than the
    one timed."""
    path = os.path.join(PROFILE_DIR, "traffic_%s_n%d.json" % (kernel, n))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if (d.get("source_hash") != kernel_source_hash(n) or d.get("variant") != variant
            or d.get("stage_form") != stage_form):
        return None
    return d.get("bytes_per_launch")


def committed_schedule(n: int, dtype: str, pad: bool):
    """The tuned schedule the committed profiles of this workload were taken
    with, if there is one."""
    if pad:
        return None
    p = os.path.join(PROFILE_DIR, "schedule_shear%d_%s.jsonl" % (n, dtype))
    return p if os.path.exists(p) else None


def plain_run(args, n, dtype, steps, warmup, profile=True, keep=False, tune=True, pad=False, retune=False):
    """Time `steps` SSP-RK3 steps of the seed-0 shear layer on one solver.
    Returns (record, final spectrum or None, dt)."""
    import torch

    from paper_2401_09843_amd import inputs, ns, perfmodel

    grid = 3 * n // 2 if pad else n  # points per axis of the passes and the physical field
    dt_torch = torch.float32 if dtype == "fp32" else torch.float64
    rbytes = 4 if dtype == "fp32" else 8
    dev = torch.device("cuda", 0)
    log("n=%d %s steps=%d warmup=%d%s" % (n, dtype, steps, warmup, " (padded to %d)" % grid if pad else ""))
    # Start from the schedule the committed profiles were taken with (a copy,
    # so that a retune on another device does not append to it); the
    # autotuner runs if its key does not match.
    cache, schedule_source = args.tune_cache, "autotuner" if tune else "built-in"
    committed = committed_schedule(n, dtype, pad)
    if cache is None and tune and not retune and committed:
        import shutil
        import tempfile
        fd, cache = tempfile.mkstemp(suffix=".jsonl")
        os.close(fd)
        shutil.copyfile(committed, cache)
        schedule_source = os.path.relpath(committed, ROOT)
    S = ns.Solver(n, dtype=dt_torch, graph=True, tune=tune, tune_cache=cache, fuse=fuse_arg(args), pad=pad)
    report = S.tune_report()
    schedule = {r["pass"]: r["selected"] for r in report}
    fused = [r for r in report if r["pass"] == "F3_fwd_z_epilogue"][0]["fused"]
    if schedule_source not in ("autotuner", "built-in"):
        with open(committed) as f:
            pinned = {d["pass"]: d["variant"] for d in map(json.loads, f)}
        form = pinned.pop("stage_form", None)
        if pinned != schedule or form != ("fused" if fused else "plain"):
            schedule_source = "autotuner"
        os.remove(cache)
    log("schedule %s" % json.dumps(report))
    u0, _, _ = inputs.shear_layer_torch(grid, seed=0, device=dev, dtype=dt_torch)
    dt = float(0.5 * (2.0 * math.pi / grid) / u0.abs().sum(dim=0).max().item())
    uh = S.forward(u0)
    del u0
    torch.cuda.synchronize()
    log("initial state ready, dt=%.3e" % dt)
    if warmup > 0:
        S.step(uh, dt, warmup)
    # the per-pass HIP events are recorded on the library's stream inside the
    # timed region itself (the profiler launches the passes eagerly instead
    # of replaying the step graph)
    if profile:
        S.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(uh, dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / steps * 1e3
    log("timed %.3f s, %.2f ms/step" % (wall, ms_per_step))
    roofline, per_pass = None, {}
    if profile:
        prof = S.profile_read()
        S.profile(False)
        bpl = perfmodel.pass_bytes_per_launch(grid, rbytes, fused=fused)
        for name, (ms, cnt) in prof.items():
            if cnt:
                avg = ms / cnt
                per_pass[name] = {"avg_ms": avg, "launches": cnt, "GBps": bpl[name] / (avg * 1e-3) / 1e9}
        dom = max(per_pass, key=lambda k: per_pass[k]["avg_ms"] * per_pass[k]["launches"])
        ach = per_pass[dom]["GBps"]
        traffic = None if pad else measured_traffic(dom, n, schedule.get(dom), "fused" if fused else "plain")
        roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "traffic": traffic, "kernel": dom, "algorithmic_bytes_per_launch": bpl[dom]}
    step_bytes = perfmodel.step_bytes(grid, rbytes, fused=fused, steps_per_call=steps)
    finite = bool(torch.isfinite(torch.view_as_real(uh)).all().item())
    rec = {
        "value": grid ** 3 * steps / wall / 1e6,
        "ms_per_step": ms_per_step,
        "steps": steps,
        "warmup": warmup,
        "hbm_model_bytes_per_step": step_bytes,
        "step_roofline_frac": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": roofline,
        "passes": per_pass,
        "schedule": schedule,
        "schedule_source": schedule_source,
        "fused_f3_inverse_z": fused,
        "finite": finite,
        "dt": dt,
    }
    S.close()
    del S
    if not keep:
        del uh
        uh = None
    torch.cuda.empty_cache()
    return rec, uh, dt


def fp64_reference_error(n, dt, nsteps, uh32):
    """Relative L2 of an FP32 final spectrum against the FP64 solver's after
    the same nsteps steps of size dt from the FP64 field of the same seed
    (built-in schedules; this is a numerical reference, not timed)."""
    import torch

    from paper_2401_09843_amd import inputs, ns

    u0, _, _ = inputs.shear_layer_torch(n, seed=0, device=torch.device("cuda", 0), dtype=torch.float64)
    S = ns.Solver(n, dtype=torch.float64, graph=True, tune=False)
    uh64 = S.forward(u0)
    del u0
    S.step(uh64, dt, nsteps)
    S.close()
    del S
    torch.cuda.empty_cache()
    num = torch.zeros((), dtype=torch.float64, device=uh64.device)
    for c in range(3):  # component by component (an FP64 copy of the whole FP32 state is large)
        num += torch.sum(torch.abs(uh32[c].to(torch.complex128) - uh64[c]) ** 2)
    err = float(torch.sqrt(num).item() / torch.linalg.vector_norm(uh64).item())
    del uh64
    torch.cuda.empty_cache()
    return err


def ensemble_fields(family, dev):
    import torch

    from paper_2401_09843_amd import inputs

    fields, dts = [], []
    for i, n in enumerate(ENS_SIZES):
        if family == "shear":
            u, _, _ = inputs.shear_layer_torch(n, seed=1000 + i, delta=(0.01, 0.05), device=dev, dtype=torch.float32)
        elif family == "tg":
            u = torch.from_numpy(inputs.perturbed_taylor_green(n, seed=1000 + i)[0]).to(dev, torch.float32)
        else:
            u = torch.from_numpy(inputs.cylindrical_shear(n, seed=1000 + i)[0]).to(dev, torch.float32)
        fields.append(u)
        dts.append(float(0.5 * (2 * math.pi / n) / u.abs().sum(0).max().item()))
    return fields, dts


def ensemble_record(args, steps, warmup, batched_only=False, statistics=False):
    """Statistical-solution ensemble: 64 samples at 128^3 and 32 at 64^3,
    FP32, seeds 1000+i, per-sample CFL dt, batched in one context (one
    launch per pass per grid size, graph-replayed steps) against looping
    single-sample solvers over the same samples.  The baseline loop uses
    plain solvers autotuned at one sample each (their own schedules); a
    second loop on the batched schedules gives the same bits as the batched
    run and is reported beside it."""
    import tempfile

    import torch

    from paper_2401_09843_amd import ns, perfmodel

    dev = torch.device("cuda", 0)
    fields, dts = ensemble_fields(args.family, dev)
    log("ensemble: %d samples, %d steps" % (len(ENS_SIZES), steps))
    E = ns.Solver(ENS_SIZES, dtype=torch.float32, graph=True, tune=not args.no_tune, tune_cache=args.tune_cache,
                  fuse=fuse_arg(args), graph_form=args.graph_form)
    uhs = E.forward(fields)
    del fields
    init = [t.clone() for t in uhs]
    E.step(uhs, dts, warmup)
    for t, t0 in zip(uhs, init):
        t.copy_(t0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step(uhs, dts, steps)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    report = E.tune_report()
    form = {r["N"]: r["fused"] for r in report if r["pass"] == "F3_fwd_z_epilogue"}
    ens_bytes = sum(perfmodel.step_bytes(n, 4, fused=form[n], steps_per_call=steps) for n in ENS_SIZES)
    rec = {
        "metric": ENS_METRIC,
        "value": len(ENS_SIZES) / (t_batched * 200.0 / steps),
        "unit": "samples/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": t_batched / steps * 1e3,
        "family": args.family,
        "hbm_model_bytes_per_step": ens_bytes,
        "step_roofline_frac": ens_bytes / (t_batched / steps) / 1e9 / HBM_PEAK_GBS,
        "schedule": report,
    }
    f3 = [r for r in report if r["pass"] == "F3_fwd_z_epilogue"]
    if f3 and "graph_form" in f3[0]:
        rec["graph_form"] = f3[0]["graph_form"]
        rec["graph_form_ms_per_step"] = f3[0]["graph_ms"]
    if batched_only:
        return rec, E, uhs
    # the baseline: plain solvers autotuned at one sample, warmed up per size
    passes = list(perfmodel.PASSES)
    fd, cache = tempfile.mkstemp(suffix=".jsonl")
    os.close(fd)
    plain = {n: ns.Solver(n, dtype=torch.float32, graph=True, tune=not args.no_tune, tune_cache=cache,
                          fuse=fuse_arg(args)) for n in sorted(set(ENS_SIZES))}
    os.remove(cache)
    plain_sched = {n: {r["pass"]: r["selected"] for r in s.tune_report()} for n, s in plain.items()}
    for n, S in plain.items():
        S.step(init[ENS_SIZES.index(n)].clone(), dts[ENS_SIZES.index(n)], warmup)

    def loop(solvers):
        out = [t.clone() for t in init]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, n in enumerate(ENS_SIZES):
            solvers[n].step(out[i], dts[i], steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    t_loop, looped = loop(plain)
    worst_tuned = max(float(torch.linalg.vector_norm(a - b).item() / torch.linalg.vector_norm(b).item())
                      for a, b in zip(uhs, looped))
    del looped
    for S in plain.values():
        S.close()
    # the same loop on the batched schedules and stage forms: same bits
    forced = {n: ns.Solver(n, dtype=torch.float32, graph=True, tune=False, fuse=form[n])
              for n in sorted(set(ENS_SIZES))}
    for r in report:
        names = list(r["timings_ms"].keys())
        forced[r["N"]].set_variant(r["N"], passes.index(r["pass"]), names.index(r["selected"]))
    for n, S in forced.items():
        S.step(init[ENS_SIZES.index(n)].clone(), dts[ENS_SIZES.index(n)], warmup)
    t_forced, looped = loop(forced)
    bitwise = all(bool(torch.equal(a, b)) for a, b in zip(uhs, looped))
    del looped
    for S in forced.values():
        S.close()
    rec.update({
        "looped_plain_samples_per_s": len(ENS_SIZES) / (t_loop * 200.0 / steps),
        "speedup_vs_loop": t_loop / t_batched,
        "looped_plain_schedules": plain_sched,
        "max_rel_diff_batched_vs_loop": worst_tuned,
        "looped_on_batched_schedules_samples_per_s": len(ENS_SIZES) / (t_forced * 200.0 / steps),
        "speedup_vs_loop_on_batched_schedules": t_forced / t_batched,
        "batched_equals_loop_on_batched_schedules_bitwise": bitwise,
    })
    # each size group alone (same samples, same batched kernels): against
    # the batched step, whether the size groups overlap at all
    alone = {}
    for n in sorted(set(ENS_SIZES)):
        idx = [i for i, m in enumerate(ENS_SIZES) if m == n]
        Sg = ns.Solver([n] * len(idx), dtype=torch.float32, graph=True, tune=not args.no_tune,
                       tune_cache=args.tune_cache, fuse=fuse_arg(args))
        xs = [init[i].clone() for i in idx]
        Sg.step(xs, [dts[i] for i in idx], warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sg.step(xs, [dts[i] for i in idx], steps)
        torch.cuda.synchronize()
        alone[str(n)] = (time.perf_counter() - t0) / steps * 1e3
        Sg.close()
    rec["group_alone_ms_per_step"] = alone
    if statistics:
        rec.update(ensemble_statistics(E, uhs))
    return rec, E, uhs


def adjoint_record(args, steps, warmup):
    """Discrete adjoint at 128^3 FP64 (the adjoint workload): the seed-0 shear
    layer, CFL dt, graph-replayed plain steps, taped steps (the stage states
    recorded) and adjoint steps back through that tape, each timed over
    `steps` steps after `warmup`; the adjoint step's cost over a plain step
    against the byte model's 1.38."""
    import torch

    from paper_2401_09843_amd import inputs, ns, perfmodel

    n = 128
    dev = torch.device("cuda", 0)
    u, _, _ = inputs.shear_layer_torch(n, seed=0, device=dev, dtype=torch.float64)
    dt = float(0.5 * (2 * math.pi / n) / u.abs().sum(0).max().item())
    S = ns.Solver(n, dtype=torch.float64, graph=True, tune=not args.no_tune, tune_cache=args.tune_cache)
    uh0 = S.forward(u)
    del u

    def timed(fn):
        fn(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    x = uh0.clone()
    t_plain = timed(lambda k: S.step(x, dt, k))
    tape = S.new_tape(max(steps, warmup))
    x = uh0.clone()
    t_taped = timed(lambda k: S.step_taped(x, dt, k, tape))
    lam = uh0.clone()
    t_adj = timed(lambda k: S.adjoint_steps(lam, dt, tape, k))
    ok = bool(torch.isfinite(torch.view_as_real(lam)).all().item())
    fb, ab = perfmodel.step_bytes(n, 8), perfmodel.adjoint_step_bytes(n, 8)
    S.close()
    return {
        "workload": "discrete adjoint, shear layer 128^3 FP64, CFL 0.5",
        "steps": steps, "warmup": warmup,
        "plain_ms_per_step": t_plain, "taped_ms_per_step": t_taped, "adjoint_ms_per_step": t_adj,
        "adjoint_over_plain": t_adj / t_plain,
        "adjoint_over_plain_bytes_model": ab / fb,
        "adjoint_step_roofline_frac": ab / (t_adj * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "plain_step_roofline_frac": fb / (t_plain * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "finite": ok,
    }


def ensemble_statistics(E, uhs):
    """In-situ statistics of the final ensemble: mean energy and enstrophy
    spectra, pointwise mean / variance over the 64 samples at 128^3,
    structure functions and the distance between the 1-point marginals of
    the two halves of the 128^3 group."""
    import torch

    kb = 112
    spec = E.spectrum(uhs, kb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zspec = E.enstrophy_spectrum(uhs, kb)
    torch.cuda.synchronize()
    t_z = time.perf_counter() - t0
    t0 = time.perf_counter()
    mom_mean, mom_var = E.moments(uhs, 128)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    t0 = time.perf_counter()
    sf2 = E.structure_functions(uhs, 16, 2.0)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    phys = torch.stack(E.inverse(uhs)[:64])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, w1_mean = E.wasserstein1(phys[:32].contiguous(), phys[32:].contiguous())
    torch.cuda.synchronize()
    t_w = time.perf_counter() - t0
    del phys
    return {
        "mean_E_k_128": spec[:64].mean(0).cpu().tolist()[:44],
        "mean_E_k_64": spec[64:].mean(0).cpu().tolist()[:38],
        "mean_Z_k_128": zspec[:64].mean(0).cpu().tolist()[:44],
        "statistics": {"enstrophy_spectra_ms": t_z * 1e3, "moments_128_ms": t_m * 1e3,
                       "rms_of_mean_128": float(mom_mean.pow(2).mean().sqrt().item()),
                       "mean_of_variance_128": float(mom_var.mean().item()),
                       "w1_halves_128_ms": t_w * 1e3, "w1_halves_128_mean": w1_mean.cpu().tolist(),
                       "structure_functions_ms": t_s * 1e3,
                       "mean_S2_128": sf2[:64].mean(0).cpu().tolist()},
    }


def run_ensemble(args):
    rec, E, uhs = ensemble_record(args, args.steps, args.warmup, batched_only=args.batched_only,
                                  statistics=not args.batched_only)
    out = {"metric": ENS_METRIC, "value": rec.pop("value"), "unit": "samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": {"shear": "synthetic: seeded shear layers, seeds 1000+i, delta ~ U[0.01,0.05]",
                    "tg": "synthetic: perturbed Taylor-Green vortices (Sec. 6.1), seeds 1000+i",
                    "cyl": "synthetic: cylindrical shear flows, sharp interface (Sec. 6.2), seeds 1000+i"}[args.family],
           "config": {"workload": "ensemble 64x128^3 + 32x64^3 FP32", "family": args.family,
                      "parallelism": "single GPU"}}
    rec.pop("metric")
    out.update(rec)
    if args.batched_only:
        out["batched_only"] = True
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 200 with --ensemble)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--only-headline", action="store_true",
                    help="the 1024^3 line alone: no FP64 check, 512^3 record, ensemble or CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in schedules instead of the autotuner")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON lines) to read or append")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner instead of starting from a committed schedule")
    ap.add_argument("--no-fuse", action="store_true",
                    help="run every stage as the plain five passes (no fused F3 + inverse z pass)")
    ap.add_argument("--fuse", action="store_true", help="end every stage in the fused F3 + inverse z pass")
    ap.add_argument("--pad", action="store_true",
                    help="Algorithm 2 in its padded form: --n modes per axis, passes on the 3n/2 grid")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--ensemble", action="store_true", help="run the 96-sample ensemble workload alone")
    ap.add_argument("--adjoint", action="store_true",
                    help="time plain, taped and adjoint steps at 128^3 FP64 (the adjoint workload) alone")
    ap.add_argument("--graph-form", default=None, choices=["chain", "branches"],
                    help="ensemble: launch the size groups of the captured step as one chain or as concurrent "
                         "graph branches (default: the autotuner's choice)")
    ap.add_argument("--batched-only", action="store_true",
                    help="with --ensemble: time the batched steps only (no looped solvers, no statistics)")
    ap.add_argument("--family", default="shear", choices=["shear", "tg", "cyl"],
                    help="initial data of the ensemble: shear layers, or the paper's perturbed Taylor-Green "
                         "vortices or cylindrical shear flows")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 2 GiB three times (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        src = torch.ones(512 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": src.numel() * 4, "bytes_written": dst.numel() * 4, "launches": 3}))
        return

    if args.steps is None:
        args.steps = 200 if args.ensemble else 20
    if args.ensemble:
        run_ensemble(args)
        return
    if args.adjoint:
        torch.cuda.set_device(torch.device("cuda", 0))
        print(json.dumps(adjoint_record(args, args.steps, args.warmup)))
        return

    torch.cuda.set_device(torch.device("cuda", 0))
    n = args.n
    grid = 3 * n // 2 if args.pad else n
    headline = n == 1024 and args.dtype == "fp32" and not args.pad
    extras = headline and not args.only_headline
    rec, uh, dt = plain_run(args, n, args.dtype, args.steps, args.warmup, profile=not args.no_profile, keep=extras,
                            tune=not args.no_tune, pad=args.pad, retune=args.retune)
    out = {
        "metric": ("Mpts*RK-steps/s (SSP-RK3, spectral hyperviscosity NS, 2/3 dealiased)" if not args.pad else
                   "Mpts*RK-steps/s (SSP-RK3, spectral hyperviscosity NS, padded 3/2; pts of the padded grid)"),
        "value": rec.pop("value"),
        "unit": "Mpts*RK-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "fp32" else "f64",
        "data": "synthetic: seeded perturbed doubly periodic shear layer (rho=0.05, delta=0.025, 16 modes |k|<=4)",
        "config": ({"workload": "shear-layer SSP-RK3 N=%d^3 %s, CFL 0.5, s=1.5, m_N=N/3" % (n, args.dtype),
                    "N": n, "parallelism": "single GPU"} if not args.pad else
                   {"workload": "shear-layer SSP-RK3, %d modes per axis padded to %d^3 (Algorithm 2) %s, "
                                "CFL 0.5 on the padded grid, s=1.5, m_N=n/3" % (n, grid, args.dtype),
                    "modes": n, "grid": grid, "parallelism": "single GPU"}),
    }
    rec.pop("steps")
    rec.pop("warmup")
    out.update(rec)
    if extras:
        log("fp64 reference of the timed run")
        out["fp32_vs_fp64"] = {"rel_l2": fp64_reference_error(n, dt, args.warmup + args.steps, uh),
                               "steps": args.warmup + args.steps, "n": n,
                               "reference": "FP64 solver on the GPU, same seed, dt and steps (built-in schedules); "
                                            "the FP64 path matches the oracle to 1e-12 per RHS"}
        del uh
        torch.cuda.empty_cache()
        log("512^3 record")
        r512, _, _ = plain_run(args, 512, "fp32", args.steps, args.warmup, profile=not args.no_profile,
                               tune=not args.no_tune)
        r512["workload"] = "shear-layer SSP-RK3 N=512^3 fp32, CFL 0.5, s=1.5, m_N=N/3"
        r512["unit"] = "Mpts*RK-steps/s"
        out["n512"] = r512
        log("ensemble record")
        ens, E, uhs = ensemble_record(args, 200, args.warmup)
        E.close()
        del E, uhs
        torch.cuda.empty_cache()
        out["ensemble"] = ens
    if not args.no_cpu_baseline and not args.pad and not args.only_headline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
