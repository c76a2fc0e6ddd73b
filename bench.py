"""Benchmark: chi^2 + gradient evaluations of the full RIME on one MI355X.

Workload (default): 64 antennas (2016 baselines), 100 timesteps, 64 channels
over 0.9-1.7 GHz, 1000 point + 500 Gaussian sources, cos^3 beam with pointing
errors and diagonal gains; observed data = model at 1 %-perturbed parameters
plus complex Gaussian noise (sigma 0.01 Jy), weights 1/sigma^2.  All inputs are
seeded synthetic data resident in HBM before the timed region.

One step = one chi^2 + gradient evaluation (every stage of the path: per-source
preparation, per-antenna phase/beam, brightness, Gaussian shape, source-summed
accumulation, fused chi^2 and the adjoint) in FP32-mixed precision.  The JSON
line also carries the FP64 figures on the same workload, the chi^2-only
figures, the roofline of the dominant kernel (timed live with HIP events on its
stream) and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks (dense): FP32 vector 157.3 TFLOP/s, FP64 vector 78.6.
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}

# Algorithmic flops per source x visibility term (4 correlations), minimal
# formulation: forward point 22, forward Gaussian 25 (+1 exp); adjoint point
# 61, adjoint Gaussian 89 (+1 exp).  The O(antennas) per-antenna work is not
# counted.
FLOPS_FWD = {"p": 22, "g": 25}
FLOPS_ADJ = {"p": 61, "g": 89}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--modes", default="grad_mixed,grad_fp64,chi2_mixed,chi2_fp64",
                    help="comma list of timed evaluations (the first must be grad_mixed)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB copied device-to-device once before timing (a kernel of known "
                         "traffic for calibrating HBM counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(name: str, seconds_target: float = 15.0):
    """Time the CPU oracle (chi^2 + autograd gradient) on a bounded sample of
    the workload: the first timestep and the first nc channels, all baselines
    and all sources, nc grown from 8 until the sample takes about
    `seconds_target` seconds.  Returns terms/s."""
    import torch

    import oracle.rime_oracle as O
    from rime_synth import make_problem

    ncores = min(os.cpu_count() or 1, 16)
    torch.set_num_threads(ncores)
    nc = 8
    while True:
        pr = make_problem(name, ntime=1, nchan=nc)
        obs, sky = pr.obs, pr.sky
        D = O.model_vis(obs, pr.truth) + pr.noise
        t0 = time.perf_counter()
        O.chi2_and_grad(obs, sky, D, pr.weight, src_chunk=32)
        dt = time.perf_counter() - t0
        full = make_problem_nchan(name)
        if dt >= seconds_target / 3 or nc >= full:
            break
        nc = min(full, int(nc * seconds_target / max(dt, 1e-3)) + 1)
    terms = obs.ntime * obs.nbl * obs.nchan * sky.nsrc
    return {"value": terms / dt, "unit": "terms/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{name} restricted to 1 timestep x {nc} channels (all {obs.nbl} "
                      f"baselines, {sky.nsrc} sources): chi2 + autograd gradient, {dt:.1f} s"}


def kernel_source_digest():
    """sha256 over the kernel sources: the HBM counters below are only valid
    for the exact code they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("rime_kernels.hip", "rime_internal.h"):
        with open(os.path.join(ROOT, "paper_1501_07719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, variant):
    """HBM bytes per launch of the timed kernel, from the committed
    FETCH_SIZE + WRITE_SIZE counter summary; None when that summary was taken
    on other kernel sources or another variant."""
    try:
        with open(path) as f:
            tr = json.load(f)
    except (OSError, ValueError):
        return None
    if tr.get("kernel_source_sha256") != kernel_source_digest() or tr.get("variant") != variant:
        return None
    return tr.get("grad_mixed_bytes_per_launch")


def make_problem_nchan(name):
    from rime_synth import CONFIGS
    return CONFIGS[name]["nchan"]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1501_07719_amd as R
    from rime_synth import make_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    name = "c1" if args.config == "c2" else args.config
    t_gen = time.perf_counter()
    pr = make_problem(name)
    obs, sky, truth = pr.obs, pr.sky, pr.truth
    log(f"generated {name}: na={obs.na} nbl={obs.nbl} ntime={obs.ntime} nchan={obs.nchan} "
        f"nsrc={sky.nsrc} in {time.perf_counter() - t_gen:.1f}s")
    plan = R.Plan(obs)
    shp = (obs.ntime, obs.nbl, obs.nchan, 4)
    # observed data: FP64 model at the truth parameters (GPU predict) + noise
    vis = torch.empty(shp, dtype=torch.complex128, device="cuda")
    ws = R.workspace(plan, R.MODE_PREDICT, R.FP64, 1, truth.nsrc)
    R.rime_predict(plan, R.DeviceSky.from_host(truth), R.FP64, vis, ws)
    D64 = vis + torch.as_tensor(pr.noise, device="cuda")
    del vis, ws
    W64 = torch.as_tensor(pr.weight, device="cuda")
    D32, W32 = D64.to(torch.complex64), W64.to(torch.float32)
    dsky = R.DeviceSky.from_host(sky)
    torch.cuda.synchronize()
    if args.calib_copy:
        # a plain device copy of known size: args.calib_copy MiB read + written
        a = torch.ones(args.calib_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    terms = obs.ntime * obs.nbl * obs.nchan * sky.nsrc
    tp = obs.ntime * obs.nbl * obs.nchan * sky.npsrc
    tg = obs.ntime * obs.nbl * obs.nchan * sky.ngsrc

    tuned = {}

    def run(mode, prec, steps, warmup):
        D, W = (D64, W64) if prec == R.FP64 else (D32, W32)
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        wsp = R.workspace(plan, mode, prec, 1, sky.nsrc)
        if not args.no_autotune:
            # untimed: the library's autotuner picks the kernel variant
            R.rime_autotune(plan, dsky, mode, prec, D, W, wsp)
        tuned[(mode, prec)] = R.rime_variant_info(mode, prec, plan.get_variant(mode, prec))

        def call():
            if mode == R.MODE_CHI2_GRAD:
                R.rime_chi2_grad(plan, dsky, prec, D, W, chi2, grad, wsp)
            else:
                R.rime_chi2(plan, dsky, prec, D, W, chi2, wsp)

        for _ in range(warmup):
            call()
        torch.cuda.synchronize()
        ks = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ke = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        for e in ks + ke:
            e.record()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for i in range(steps):
            plan.set_timing_events(ks[i], ke[i])
            call()
        stop.record()
        torch.cuda.synchronize()
        plan.set_timing_events(None, None)
        ms = start.elapsed_time(stop) / steps
        kms = float(np.mean([ks[i].elapsed_time(ke[i]) for i in range(steps)]))
        return {"ms_per_step": ms, "kernel_ms": kms, "chi2": chi2.item(),
                "variant": tuned[(mode, prec)],
                "terms_per_s": terms / (ms * 1e-3), "evals_per_s": 1e3 / ms}

    out = {}
    modes = [m for m in args.modes.split(",") if m]
    if args.no_fp64:
        modes = [m for m in modes if not m.endswith("fp64")]
    spec = {"grad_mixed": (R.MODE_CHI2_GRAD, R.MIXED, args.steps, args.warmup),
            "grad_fp64": (R.MODE_CHI2_GRAD, R.FP64, max(2, args.steps // 2), 1),
            "chi2_mixed": (R.MODE_CHI2, R.MIXED, args.steps, 1),
            "chi2_fp64": (R.MODE_CHI2, R.FP64, max(2, args.steps // 2), 1)}
    for m in modes:
        log("timing", m)
        out[m] = run(*spec[m])
        log(m, out[m])

    g = out["grad_mixed"]
    flops = tp * (FLOPS_FWD["p"] + FLOPS_ADJ["p"]) + tg * (FLOPS_FWD["g"] + FLOPS_ADJ["g"])
    achieved = flops / (g["kernel_ms"] * 1e-3) / 1e12
    traffic = measured_traffic(args.traffic, list(g["variant"]))
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f32"],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f32"], "traffic": traffic,
                "kernel": "rime_main<float, %d, %d, %d, chi2+grad>" % tuple(g["variant"]),
                "kernel_ms": g["kernel_ms"],
                "flops_per_launch": flops}
    rec = {
        "metric": "source x visibility terms/s (chi2+grad, FP32-mixed), 1 GPU",
        "value": g["terms_per_s"],
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: RIME chi2+grad, {obs.na} antennas ({obs.nbl} "
                               f"baselines), {obs.ntime} timesteps, {obs.nchan} channels, "
                               f"{sky.npsrc} point + {sky.ngsrc} Gaussian sources, beam",
                   "terms_per_eval": terms, "precision": "mixed (FP64 phase and sums)"},
        "evals_per_s": g["evals_per_s"],
        "roofline": roofline,
    }
    if "grad_fp64" in out:
        rec["fp64"] = {"terms_per_s": out["grad_fp64"]["terms_per_s"],
                       "ms_per_step": out["grad_fp64"]["ms_per_step"],
                       "evals_per_s": out["grad_fp64"]["evals_per_s"]}
        rec["speedup_mixed_vs_fp64"] = out["grad_fp64"]["ms_per_step"] / g["ms_per_step"]
    if "chi2_mixed" in out and "chi2_fp64" in out:
        rec["chi2_only"] = {
            "mixed_terms_per_s": out["chi2_mixed"]["terms_per_s"],
            "fp64_terms_per_s": out["chi2_fp64"]["terms_per_s"],
            "mixed_ms": out["chi2_mixed"]["ms_per_step"],
            "fp64_ms": out["chi2_fp64"]["ms_per_step"]}
    if not args.no_cpu_baseline:
        log("cpu baseline")
        rec["cpu_baseline"] = cpu_baseline(name)
    plan.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
