"""Benchmark: SSP-RK3 steps of the spectral hyperviscosity solver on one MI355X.

Default workload: the seeded perturbed shear layer at N = 1024^3, FP32, s = 1.5,
step multiplier at m_N = N/3, eps_N = 1e-3 (32/N)^2, dt from CFL 0.5; W warm-up
steps (graph replay), then K timed steps in one ns_step call, inputs resident
in HBM.  A stage runs the plain five passes or, in the fused form, four (the
forward z pass also writes the inverse z transform of the new state); the
autotuner picks the faster form (--fuse / --no-fuse force one).  The
timed steps run with the pass profiler on: HIP events bracket every pass
launch on the library's stream (eager launches; --no-profile times graph
replays instead).  Prints one JSON line with Mpts*RK-steps/s,
the HBM roofline of the dominant pass (algorithmic bytes / its average
event-timed duration in the timed region) and the CPU oracle timed on a
bounded sample of the same workload family.

    python bench.py [--gpus 1] [--steps 20] [--warmup 2] [--n 1024]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def cpu_baseline(n_sample: int = 256):
    """The oracle (FP64, all host cores) for one SSP-RK3 step of the same
    shear-layer family at n_sample^3; returns Mpts*RK-steps/s."""
    from oracle import oracle as orc
    from paper_2401_09843_amd import inputs

    u0, _, _ = inputs.shear_layer(n_sample, seed=0)
    dt = inputs.cfl_dt(u0)
    uh = orc.initial_state(u0)
    t0 = time.perf_counter()
    orc.ssprk3(uh, n_sample, dt, 1)
    t = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_sample ** 3 / t / 1e6, "unit": "Mpts*RK-steps/s", "cores": cores, "kind": "oracle",
            "sample": "one SSP-RK3 step (3 RHS) of the seed-0 shear layer at %d^3, FP64, %.1f s" % (n_sample, t)}


def run_ensemble(args):
    """Statistical-solution ensemble: 64 samples at 128^3 and 32 at 64^3,
    FP32, seeds 1000+i, delta ~ U[0.01, 0.05], per-sample CFL dt, batched in
    one context (one launch per pass per grid size, graph-replayed steps)
    against looping single-sample solvers over the same samples."""
    import torch

    from paper_2401_09843_amd import inputs, ns

    steps = args.steps
    sizes = [128] * 64 + [64] * 32
    dev = torch.device("cuda", 0)
    fields, dts = [], []
    for i, n in enumerate(sizes):
        if args.family == "shear":
            u, _, _ = inputs.shear_layer_torch(n, seed=1000 + i, delta=(0.01, 0.05), device=dev, dtype=torch.float32)
        elif args.family == "tg":
            u = torch.from_numpy(inputs.perturbed_taylor_green(n, seed=1000 + i)[0]).to(dev, torch.float32)
        else:
            u = torch.from_numpy(inputs.cylindrical_shear(n, seed=1000 + i)[0]).to(dev, torch.float32)
        fields.append(u)
        dts.append(float(0.5 * (2 * 3.141592653589793 / n) / u.abs().sum(0).max().item()))
    print("ensemble: %d samples, %d steps" % (len(sizes), steps), file=sys.stderr, flush=True)
    E = ns.Solver(sizes, dtype=torch.float32, graph=True, tune=not args.no_tune, tune_cache=args.tune_cache,
                  fuse=fuse_arg(args))
    uhs = E.forward(fields)
    init = [t.clone() for t in uhs]
    E.step(uhs, dts, args.warmup)
    for t, t0 in zip(uhs, init):
        t.copy_(t0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step(uhs, dts, steps)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    if args.batched_only:  # the batched steps alone (for a kernel trace)
        print(json.dumps({"metric": "ensemble samples/s (96 samples: 64x128^3 + 32x64^3, 200 SSP-RK3 steps)",
                          "value": len(sizes) / (t_batched * 200.0 / steps), "unit": "samples/s", "n_gpus": 1,
                          "steps": steps, "warmup": args.warmup, "ms_per_step": t_batched / steps * 1e3,
                          "family": args.family, "batched_only": True, "schedule": E.tune_report()}))
        return
    # looping the plain solver (one context per grid size, one sample at a time)
    # with the schedules the ensemble runs, so that both compute the same bits
    form = {r["N"]: r["fused"] for r in E.tune_report() if r["pass"] == "F3_fwd_z_epilogue"}
    plain = {n: ns.Solver(n, dtype=torch.float32, graph=True, tune=False, fuse=form[n]) for n in sorted(set(sizes))}
    passes = ["I1_inv_z", "I2_inv_y", "X_c2r_prod_r2c", "F2_fwd_y", "F3_fwd_z_epilogue"]
    for r in E.tune_report():
        names = list(r["timings_ms"].keys())
        plain[r["N"]].set_variant(r["N"], passes.index(r["pass"]), names.index(r["selected"]))
    loop = [t.clone() for t in init]
    for i, n in enumerate(sizes[:2]):
        plain[n].step(init[i].clone(), dts[i], args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, n in enumerate(sizes):
        plain[n].step(loop[i], dts[i], steps)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    worst = 0.0
    for a, b in zip(uhs, loop):
        d = torch.linalg.vector_norm(a - b).item() / torch.linalg.vector_norm(b).item()
        worst = max(worst, d)
    kb = 112
    spec = E.spectrum(uhs, kb)
    mean128 = spec[:64].mean(0).cpu().tolist()
    mean64 = spec[64:].mean(0).cpu().tolist()
    # in-situ statistics of the final ensemble: enstrophy spectra and the
    # pointwise mean / variance over the 64 samples at 128^3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zspec = E.enstrophy_spectrum(uhs, kb)
    torch.cuda.synchronize()
    t_z = time.perf_counter() - t0
    t0 = time.perf_counter()
    mom_mean, mom_var = E.moments(uhs, 128)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    zmean128 = zspec[:64].mean(0).cpu().tolist()
    t0 = time.perf_counter()
    sf2 = E.structure_functions(uhs, 16, 2.0)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    # distance between the 1-point marginals of the two halves of the 128^3 group
    phys = torch.stack(E.inverse(uhs)[:64])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, w1_mean = E.wasserstein1(phys[:32].contiguous(), phys[32:].contiguous())
    torch.cuda.synchronize()
    t_w = time.perf_counter() - t0
    del phys
    out = {
        "metric": "ensemble samples/s (96 samples: 64x128^3 + 32x64^3, 200 SSP-RK3 steps)",
        "value": len(sizes) / (t_batched * 200.0 / steps),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": t_batched / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": {"shear": "synthetic: seeded shear layers, seeds 1000+i, delta ~ U[0.01,0.05]",
                 "tg": "synthetic: perturbed Taylor-Green vortices (Sec. 6.1), seeds 1000+i",
                 "cyl": "synthetic: cylindrical shear flows, sharp interface (Sec. 6.2), seeds 1000+i"}[args.family],
        "config": {"workload": "ensemble 64x128^3 + 32x64^3 FP32", "family": args.family,
                   "parallelism": "single GPU"},
        "looped_plain_samples_per_s": len(sizes) / (t_loop * 200.0 / steps),
        "speedup_vs_loop": t_loop / t_batched,
        "max_rel_diff_batched_vs_loop": worst,
        "mean_E_k_128": mean128[:44],
        "mean_E_k_64": mean64[:38],
        "mean_Z_k_128": zmean128[:44],
        "statistics": {"enstrophy_spectra_ms": t_z * 1e3, "moments_128_ms": t_m * 1e3,
                       "rms_of_mean_128": float(mom_mean.pow(2).mean().sqrt().item()),
                       "mean_of_variance_128": float(mom_var.mean().item()),
                       "w1_halves_128_ms": t_w * 1e3, "w1_halves_128_mean": w1_mean.cpu().tolist(),
                       "structure_functions_ms": t_s * 1e3,
                       "mean_S2_128": sf2[:64].mean(0).cpu().tolist()},
        "schedule": E.tune_report(),
    }
    print(json.dumps(out))


def fuse_arg(args):
    """Stage form requested on the command line: None lets the autotuner
    choose."""
    if args.fuse and args.no_fuse:
        sys.exit("--fuse and --no-fuse exclude each other")
    return True if args.fuse else (False if args.no_fuse else None)


def kernel_source_hash() -> str:
    """SHA-256 of the HIP sources; PMC traffic figures are valid only for
    the kernels they were measured on."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2401_09843_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, n: int, variant: str):
    """HBM bytes per launch of a pass from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None if there is none, the kernels changed since, or
    the figure belongs to another schedule variant than the one timed."""
    path = os.path.join(PROFILE_DIR, "traffic_%s_n%d.json" % (kernel, n))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash() or d.get("variant") != variant:
        return None
    return d.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 200 with --ensemble)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in schedules instead of the autotuner")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON lines) to read or append")
    ap.add_argument("--retune", action="store_true",
                    help="at 1024^3 FP32, run the autotuner instead of starting from the committed schedule")
    ap.add_argument("--no-fuse", action="store_true",
                    help="run every stage as the plain five passes (no fused F3 + inverse z pass)")
    ap.add_argument("--fuse", action="store_true", help="end every stage in the fused F3 + inverse z pass")
    ap.add_argument("--pad", action="store_true",
                    help="Algorithm 2 in its padded form: --n modes per axis, passes on the 3n/2 grid")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--ensemble", action="store_true", help="run the 96-sample ensemble workload instead")
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

    from paper_2401_09843_amd import inputs, ns, perfmodel

    n = args.n
    grid = 3 * n // 2 if args.pad else n  # points per axis of the passes and the physical field
    dt_torch = torch.float32 if args.dtype == "fp32" else torch.float64
    rbytes = 4 if args.dtype == "fp32" else 8
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print("bench: n=%d %s steps=%d warmup=%d" % (n, args.dtype, args.steps, args.warmup), file=sys.stderr, flush=True)

    # At 1024^3 FP32 the solver starts from the schedule the committed
    # profiles were taken with (a copy, so that a retune on another device
    # does not append to it); the autotuner runs if its key does not match.
    cache, schedule_source = args.tune_cache, "autotuner"
    committed = os.path.join(PROFILE_DIR, "schedule_shear1024_fp32.jsonl")
    if cache is None and not args.retune and not args.no_tune and n == 1024 and not args.pad \
            and args.dtype == "fp32" and os.path.exists(committed):
        import shutil
        import tempfile
        fd, cache = tempfile.mkstemp(suffix=".jsonl")
        os.close(fd)
        shutil.copyfile(committed, cache)
        schedule_source = "profiles/schedule_shear1024_fp32.jsonl"
    S = ns.Solver(n, dtype=dt_torch, graph=True, tune=not args.no_tune, tune_cache=cache, fuse=fuse_arg(args),
                  pad=args.pad)
    schedule = {r["pass"]: r["selected"] for r in S.tune_report()}
    fused = [r for r in S.tune_report() if r["pass"] == "F3_fwd_z_epilogue"][0]["fused"]
    if schedule_source != "autotuner":
        with open(committed) as f:
            pinned = {d["pass"]: d["variant"] for d in map(json.loads, f)}
        form = pinned.pop("stage_form", None)
        if pinned != schedule or form != ("fused" if fused else "plain"):
            schedule_source = "autotuner"
        os.remove(cache)
    print("bench: schedule %s" % json.dumps(S.tune_report()), file=sys.stderr, flush=True)
    u0, _, _ = inputs.shear_layer_torch(grid, seed=0, device=dev, dtype=dt_torch)
    dt = float(0.5 * (2.0 * 3.141592653589793 / grid) / u0.abs().sum(dim=0).max().item())
    uh = S.forward(u0)
    del u0
    torch.cuda.synchronize()
    print("bench: initial state ready, dt=%.3e" % dt, file=sys.stderr, flush=True)

    if args.warmup > 0:
        S.step(uh, dt, args.warmup)
    # the per-pass HIP events are recorded on the library's stream inside the
    # timed region itself (the profiler launches the passes eagerly instead
    # of replaying the step graph)
    if not args.no_profile:
        S.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(uh, dt, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = wall / args.steps * 1e3
    value = grid ** 3 * args.steps / wall / 1e6
    print("bench: timed %.3f s, %.2f ms/step" % (wall, ms_per_step), file=sys.stderr, flush=True)

    roofline = None
    per_pass = {}
    if not args.no_profile:
        prof = S.profile_read()
        S.profile(False)
        bpl = perfmodel.pass_bytes_per_launch(grid, rbytes, fused=fused)
        for name, (ms, cnt) in prof.items():
            if cnt:
                avg = ms / cnt
                per_pass[name] = {"avg_ms": avg, "launches": cnt, "GBps": bpl[name] / (avg * 1e-3) / 1e9}
        dom = max(per_pass, key=lambda k: per_pass[k]["avg_ms"] * per_pass[k]["launches"])
        ach = per_pass[dom]["GBps"]
        traffic = None if args.pad else measured_traffic(dom, n, schedule.get(dom))
        roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "traffic": traffic, "kernel": dom, "algorithmic_bytes_per_launch": bpl[dom]}
    step_bytes = perfmodel.step_bytes(grid, rbytes, fused=fused, steps_per_call=args.steps)
    finite = bool(torch.isfinite(torch.view_as_real(uh)).all().item())

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    out = {
        "metric": ("Mpts*RK-steps/s (SSP-RK3, spectral hyperviscosity NS, 2/3 dealiased)" if not args.pad else
                   "Mpts*RK-steps/s (SSP-RK3, spectral hyperviscosity NS, padded 3/2; pts of the padded grid)"),
        "value": value,
        "unit": "Mpts*RK-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
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
        "hbm_model_bytes_per_step": step_bytes,
        "step_roofline_frac": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": roofline,
        "passes": per_pass,
        "schedule": schedule,
        "schedule_source": schedule_source,
        "fused_f3_inverse_z": fused,
        "finite": finite,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
