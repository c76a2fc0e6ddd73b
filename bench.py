"""Benchmark: chi^2 + gradient evaluations of the full RIME on one MI355X.

Default workload (c2): 64 antennas (2016 baselines), 100 timesteps, 64
channels over 0.9-1.7 GHz, 1000 point + 500 Gaussian sources, cos^3 beam with
pointing errors and diagonal gains.  The observed data is the model at
1 %-perturbed parameters plus complex Gaussian noise (sigma 0.01 Jy), with
weights 1/sigma^2.  All inputs are seeded synthetic data, resident in HBM
before the timed region.

One step is one chi^2 + gradient evaluation in FP32-mixed precision.  It runs
every stage of the path:
- per-source preparation;
- per-antenna phase and beam;
- brightness and Gaussian shape;
- the source-summed accumulation;
- the fused chi^2;
- the adjoint.

The JSON line also carries:
- the FP64 figures and the chi^2-only figures on the same workload;
- the roofline of the dominant kernel, timed live with HIP events on its stream;
- the CPU oracle, timed on a bounded sample of the same workload.

Other workloads (`--config`), which give the same JSON line for their own
shape:
- c0: 7 antennas, 10 t, 16 ch, 20 points, no beam, FP64.  Latency of one
  graph-launched chi^2 + gradient.
- c3: 256 proposals of 10..2000 sources over one 64-antenna observation
  (50 t, 32 ch).  Batched in one graph launch, compared with a per-set loop
  and with the default kernel variant.
- c4: 197 antennas (19306 baselines), 20 t, 256 ch, 1500 P + 500 G, beam.
- c4p: the 1500 point sources of c4, beam-free (and, for chi^2, with the
  beam), through every float32-mixed variant: the per-baseline VALU kernels
  against the antenna x antenna contraction on the matrix cores.
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

# MI355X peaks (dense).  Published: FP32 vector 157.3 TFLOP/s (with packed
# dual FP32 instructions), FP64 vector 78.6, fp16 matrix 2.5 PFLOP/s.  This
# build compiles without packed FP32 (v_pk_fma_f32 is disabled for all device
# code), so its float32 vector ceiling is the one derived from the unit
# counts and clock: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz =
# 78.6 TFLOP/s.
PEAK_TFLOPS = {"f32": 78.6, "f32_packed": 157.3, "f64": 78.6, "f16_mfma": 2500.0}

# Algorithmic flops per source x visibility term (4 correlations), minimal
# formulation: forward point 22, forward Gaussian 25 (+1 exp); adjoint point
# 61, adjoint Gaussian 89 (+1 exp).  The O(antennas) per-antenna work is not
# counted.
FLOPS_FWD = {"p": 22, "g": 25}
FLOPS_ADJ = {"p": 61, "g": 89}

# timed repetitions per workload (at least 20 where a step is short) after
# --warmup untimed ones
DEFAULT_STEPS = {"c0": 200, "c2": 20, "c3": 10, "c4": 20, "c4p": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=["c0", "c1", "c2", "c3", "c4", "c4p"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--variant", type=int, default=None,
                    help="pin the float32-mixed kernel variant (library index) instead of "
                         "autotuning it")
    ap.add_argument("--modes", default="grad_mixed,grad_res64,grad_fp64,chi2_mixed,chi2_fp64,"
                                       "grad_terms,grad_disk,grad_streamed",
                    help="comma list of timed evaluations (the first must be grad_mixed); "
                         "grad_terms, grad_disk and grad_streamed time the per-call terms, the "
                         "exponential-disk morphology and the out-of-core path")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB copied device-to-device once before timing (a kernel of known "
                         "traffic for calibrating HBM counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--write-traffic", nargs=2, action="append", metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="host only: write the --traffic summary from the counter_collection "
                         "CSVs of a FETCH_SIZE and a WRITE_SIZE rocprofv3 pass of "
                         "'bench.py --variant N --modes grad_mixed --calib-copy 1024' (one pair "
                         "per variant) for the workload given by --config, merged into an "
                         "existing summary of the same kernel sources, and exit")
    a = ap.parse_args()
    if a.config == "c1":
        a.config = "c2"
    if a.steps is None:
        a.steps = DEFAULT_STEPS[a.config]
    return a


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- #
# CPU oracle baseline (the only part of this file that runs the oracle)
# --------------------------------------------------------------------------- #

def cpu_baseline(sample_fn, seconds_target: float = 15.0):
    """Time the CPU oracle (chi^2 + autograd gradient) on a bounded sample:
    `sample_fn(nc)` returns (obs, sky, D, W, description, nchan of the full
    workload) restricted to nc channels of one timestep; nc grows from 8 until
    the sample takes about `seconds_target` seconds.  Returns the cpu_baseline
    record in terms/s."""
    import torch

    import oracle.rime_oracle as O

    # the GPU machine gives one GPU a share of 16 host cores, whatever
    # os.cpu_count() reports there
    ncores = min(os.cpu_count() or 1, 16)
    torch.set_num_threads(ncores)
    nc = 8
    while True:
        obs, sky, D, W, desc, full = sample_fn(nc)
        t0 = time.perf_counter()
        O.chi2_and_grad(obs, sky, D, W, src_chunk=32)
        dt = time.perf_counter() - t0
        if dt >= seconds_target / 3 or nc >= full:
            break
        nc = min(full, int(nc * seconds_target / max(dt, 1e-3)) + 1)
    terms = obs.ntime * obs.nbl * obs.nchan * sky.nsrc
    return {"value": terms / dt, "unit": "terms/s", "cores": torch.get_num_threads(),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{desc} restricted to 1 timestep x {nc} channels (all {obs.nbl} "
                      f"baselines, {sky.nsrc} sources): chi2 + autograd gradient, {dt:.1f} s"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def problem_sample(name):
    def fn(nc):
        import oracle.rime_oracle as O
        from rime_synth import CONFIGS, make_problem
        pr = make_problem(name, ntime=1, nchan=nc)
        D = O.model_vis(pr.obs, pr.truth) + pr.noise
        return pr.obs, pr.sky, D, pr.weight, name, CONFIGS[name]["nchan"]
    return fn


def batch_sample(pb, set_index):
    def fn(nc):
        import oracle.rime_oracle as O
        obs = pb.obs.time_slice(0, 1).chan_slice(0, nc)
        D = O.model_vis(obs, pb.truth) + pb.noise[:1, :, :nc]
        W = pb.weight[:1, :, :nc]
        return obs, pb.skies[set_index], D, W, f"c3 proposal {set_index}", pb.obs.nchan
    return fn


# --------------------------------------------------------------------------- #
# helpers
# --------------------------------------------------------------------------- #

def kernel_source_digest():
    """sha256 over the kernel sources: the HBM counters below are only valid
    for the exact code they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("rime_kernels.hip", "rime_pme.hip", "rime_device.h", "rime_internal.h"):
        with open(os.path.join(ROOT, "paper_1501_07719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, variant, workload):
    """HBM bytes per launch of the timed kernel, from the committed
    FETCH_SIZE + WRITE_SIZE counter summary (one entry per kernel variant);
    None when that summary was taken on other kernel sources, or has no entry
    for this variant and workload."""
    try:
        with open(path) as f:
            tr = json.load(f)
    except (OSError, ValueError):
        return None
    if tr.get("kernel_source_sha256") != kernel_source_digest():
        return None
    for e in tr.get("entries", []):
        if e.get("variant") == variant and e.get("workload") == workload:
            return e.get("grad_mixed_bytes_per_launch")
    return None


def alg_flops(tp, tg):
    return tp * (FLOPS_FWD["p"] + FLOPS_ADJ["p"]) + tg * (FLOPS_FWD["g"] + FLOPS_ADJ["g"])


def roofline(flops, kernel_ms, variant, traffic):
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f32"],
            "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f32"], "traffic": traffic,
            "peak_packed": PEAK_TFLOPS["f32_packed"],
            "frac_packed": achieved / PEAK_TFLOPS["f32_packed"],
            "kernel": "rime_main<float, %d, %d, %d, chi2+grad>" % tuple(variant),
            "kernel_ms": kernel_ms, "flops_per_launch": flops}


def rooflines(g, tp, tg, obs, sky, traffic, npoint=None):
    """Roofline objects of one chi^2 + gradient call.  Without the matrix
    cores the per-baseline kernel does all the work: VALU-bound, algorithmic
    flops of all terms over its time.  With them it does the Gaussian sources
    (algorithmic flops of the Gaussian terms over its time) and the point
    sources run on the matrix cores (executed fp16 MFMA flops over the time of
    those kernels, against the dense fp16 peak); the larger time is the
    dominant kernel and goes in "roofline", the other in "roofline_other"."""
    main = roofline(alg_flops(0 if g["matrix_cores"] else tp, tg), g["main_ms"], g["variant"],
                    traffic)
    main["kernel_ms"] = g["main_ms"]
    if not g["matrix_cores"]:
        return {"roofline": main}
    mc_ms = g["kernel_ms"] - g["main_ms"]
    # the method's own work on the point sources (the algorithmic flops of
    # the point terms), and what the matrix cores execute for it (three fp16
    # products per hi/lo pair, full 32 x 32 tiles)
    fl = alg_flops(tp, 0)
    ach = fl / (mc_ms * 1e-3) / 1e12
    fl_exec = mfma_flops(obs, sky.npsrc if npoint is None else npoint)
    mc = {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["f16_mfma"], "unit": "TFLOP/s",
          "frac": ach / PEAK_TFLOPS["f16_mfma"], "traffic": None,
          "kernel": "pme_phase + pme_forward + pme_mfrag + pme_adjoint (point sources)",
          "kernel_ms": mc_ms, "flops_per_launch": fl,
          "executed_mfma_flops_per_launch": fl_exec,
          "executed_tflops": fl_exec / (mc_ms * 1e-3) / 1e12}
    main["kernel"] += " (Gaussian sources)"
    if mc_ms > g["main_ms"]:
        return {"roofline": mc, "roofline_other": main}
    return {"roofline": main, "roofline_other": mc}


def timed(call, steps, warmup, events_fns=(), per_step=False):
    """Mean ms per call over `steps` timed calls after `warmup` untimed ones.
    Each of `events_fns` is a setter `fn(start, stop)` installing a pair of
    per-call timing events in the library (None, None removes it).  Returns
    (ms, [mean ms between each pair], per-call ms or None).  With `per_step`,
    a second pass of `steps` calls records an event after every call (kept
    out of the first pass, where the extra records would add to a launch-bound
    mean) and gives the per-call times."""
    import torch
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    evs = []
    for _ in events_fns:
        ks = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ke = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        # torch creates the underlying hipEvent on first record: record each
        # once so that the handles passed to the library are valid
        for e in ks + ke:
            e.record()
        evs.append((ks, ke))
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for i in range(steps):
        for fn, (ks, ke) in zip(events_fns, evs):
            fn(ks[i], ke[i])
        call()
    stop.record()
    torch.cuda.synchronize()
    for fn in events_fns:
        fn(None, None)
    ms = start.elapsed_time(stop) / steps
    kms = [float(np.mean([ks[i].elapsed_time(ke[i]) for i in range(steps)])) for ks, ke in evs]
    step_ms = None
    if per_step:
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        marks[0].record()
        for i in range(steps):
            call()
            marks[i + 1].record()
        torch.cuda.synchronize()
        step_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(steps)]
    return ms, kms, step_ms


def step_stats(step_ms):
    """Median and 10th/90th percentiles of per-call times (ms)."""
    a = np.asarray(step_ms, dtype=np.float64)
    return {"n": int(a.size), "median": float(np.median(a)),
            "p10": float(np.percentile(a, 10)), "p90": float(np.percentile(a, 90))}


def mfma_flops(obs, npsrc):
    """fp16 matrix-core flops one chi^2 + gradient call executes with a
    matrix-core variant: per (timestep, channel) and 32-source chunk, the
    forward runs 4 Stokes x 6 products x 4 K-steps per antenna-pair tile and
    the adjoint 4 x 6 x 4 per (P block, q block); 32x32x16 = 32768 flops."""
    nblk = (obs.na + 31) // 32
    pairs = {(min(a // 32, b // 32), max(a // 32, b // 32)) for a, b in zip(obs.ant1, obs.ant2)}
    # npsrc: one count, or the counts of the sets of a batch (one pipeline each)
    nch = sum((int(n) + 31) // 32 for n in np.atleast_1d(npsrc))
    per_slice = 96 * nch * (len(pairs) + nblk * nblk)
    return per_slice * obs.ntime * obs.nchan * 32768


def upload_data(R, plan, truth, noise, weight):
    """D = FP64 model at the truth parameters (GPU predict) + noise, in both
    precisions, resident on the device."""
    import torch
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    vis = torch.empty(shp, dtype=torch.complex128, device="cuda")
    ws = R.workspace(plan, R.MODE_PREDICT, R.FP64, 1, truth.nsrc)
    R.rime_predict(plan, R.DeviceSky.from_host(truth), R.FP64, vis, ws)
    vis += torch.as_tensor(noise, device="cuda")
    del ws
    W64 = torch.as_tensor(weight, device="cuda")
    D32, W32 = vis.to(torch.complex64), W64.to(torch.float32)
    torch.cuda.synchronize()
    return vis, W64, D32, W32


def calib_copy(mib):
    import torch
    if mib:
        # a plain device copy of known size: mib MiB read + written; then a
        # sum over the same mib MiB (read only), a second access mix for the
        # FETCH_SIZE factor
        a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del b
        a.sum()
        torch.cuda.synchronize()
        del a


MIXED_PRECISION = "float32 per term; FP64 phase argument, chi2 and gradient sums"
MIXED_PRECISION_MC = (MIXED_PRECISION + "; point-source products on the matrix cores from "
                      "fp16 hi + lo operands (hi*hi + hi*lo + lo*hi, about 22 bits)")


def base_record(args, metric, value, ms, dtype, workload, extra_cfg):
    cfg = {"workload": workload}
    cfg.update(extra_cfg)
    return {"metric": metric, "value": value, "unit": "terms/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": cfg}


# --------------------------------------------------------------------------- #
# single-sky workloads: c2 (default) and c4
# --------------------------------------------------------------------------- #

def bench_single(args):
    import torch

    import paper_1501_07719_amd as R
    from rime_synth import make_problem

    name = "c1" if args.config == "c2" else args.config
    t_gen = time.perf_counter()
    pr = make_problem(name)
    obs, sky, truth = pr.obs, pr.sky, pr.truth
    log(f"generated {name}: na={obs.na} nbl={obs.nbl} ntime={obs.ntime} nchan={obs.nchan} "
        f"nsrc={sky.nsrc} in {time.perf_counter() - t_gen:.1f}s")
    plan = R.Plan(obs)
    D64, W64, D32, W32 = upload_data(R, plan, truth, pr.noise, pr.weight)
    del pr
    dsky = R.DeviceSky.from_host(sky)
    calib_copy(args.calib_copy)

    terms = obs.ntime * obs.nbl * obs.nchan * sky.nsrc
    tp = obs.ntime * obs.nbl * obs.nchan * sky.npsrc
    tg = obs.ntime * obs.nbl * obs.nchan * sky.ngsrc
    # FP64 autotuning at the large array would take longer than the timing
    tune_fp64 = args.config != "c4"

    def run(mode, prec, steps, warmup):
        D, W = (D64, W64) if prec == R.FP64 else (D32, W32)
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        wsp = R.workspace(plan, mode, prec, 1, sky.nsrc)
        if prec == R.MIXED and args.variant is not None:
            plan.set_variant(mode, prec, args.variant)
        elif not args.no_autotune and (prec != R.FP64 or tune_fp64):
            # untimed: the library's autotuner picks the kernel variant
            R.rime_autotune(plan, dsky, mode, prec, D, W, wsp)
        variant = R.rime_variant_info(mode, prec, plan.get_variant(mode, prec))

        def call():
            if mode == R.MODE_CHI2_GRAD:
                R.rime_chi2_grad(plan, dsky, prec, D, W, chi2, grad, wsp)
            else:
                R.rime_chi2(plan, dsky, prec, D, W, chi2, wsp)

        ms, (kms, mms), step_ms = timed(call, steps, warmup,
                                        (plan.set_timing_events, plan.set_main_events),
                                        per_step=True)
        mc = R.rime_variant_matrix_cores(mode, prec, plan.get_variant(mode, prec))
        return {"ms_per_step": ms, "step_ms": step_stats(step_ms), "kernel_ms": kms,
                "main_ms": mms, "chi2": chi2.item(),
                "variant": variant, "matrix_cores": mc,
                "terms_per_s": terms / (ms * 1e-3), "evals_per_s": 1e3 / ms}

    out = {}
    modes = [m for m in args.modes.split(",") if m]
    if args.no_fp64:
        modes = [m for m in modes if not m.endswith("fp64")]

    fp_steps = max(2, args.steps // 2)
    spec = {"grad_mixed": (R.MODE_CHI2_GRAD, R.MIXED, args.steps, args.warmup),
            "grad_fp64": (R.MODE_CHI2_GRAD, R.FP64, fp_steps, 1),
            "chi2_mixed": (R.MODE_CHI2, R.MIXED, args.steps, 1),
            "chi2_fp64": (R.MODE_CHI2, R.FP64, fp_steps, 1),
            "grad_res64": (R.MODE_CHI2_GRAD, R.MIXED_RES64, args.steps, 1)}
    for m in modes:
        if m not in spec:
            continue  # the timings of bench_extras
        log("timing", m)
        out[m] = run(*spec[m])
        log(m, out[m])

    g = out["grad_mixed"]
    traffic = measured_traffic(args.traffic, list(g["variant"]) + [int(g["matrix_cores"])],
                               args.config)
    rec = base_record(
        args, "source x visibility terms/s (chi2+grad, FP32-mixed), 1 GPU", g["terms_per_s"],
        g["ms_per_step"], "f32",
        f"{args.config}: RIME chi2+grad, {obs.na} antennas ({obs.nbl} baselines), "
        f"{obs.ntime} timesteps, {obs.nchan} channels, {sky.npsrc} point + {sky.ngsrc} "
        f"Gaussian sources, beam",
        {"terms_per_eval": terms,
         "precision": MIXED_PRECISION_MC if g["matrix_cores"] else MIXED_PRECISION})
    rec["evals_per_s"] = g["evals_per_s"]
    rec["step_ms"] = g["step_ms"]
    rec["variant"] = {"per_baseline": list(g["variant"]), "matrix_cores": g["matrix_cores"]}
    rec.update(rooflines(g, tp, tg, obs, sky, traffic))
    if "grad_fp64" in out:
        rec["fp64"] = {"terms_per_s": out["grad_fp64"]["terms_per_s"],
                       "ms_per_step": out["grad_fp64"]["ms_per_step"],
                       "evals_per_s": out["grad_fp64"]["evals_per_s"],
                       "variant": out["grad_fp64"]["variant"]}
        rec["speedup_mixed_vs_fp64"] = out["grad_fp64"]["ms_per_step"] / g["ms_per_step"]
    if "grad_res64" in out:
        r64 = out["grad_res64"]
        rec["res64"] = {"terms_per_s": r64["terms_per_s"], "ms_per_step": r64["ms_per_step"],
                        "step_ms": r64["step_ms"], "evals_per_s": r64["evals_per_s"],
                        "variant": r64["variant"], "matrix_cores": r64["matrix_cores"],
                        "main_ms": r64["main_ms"], "kernel_ms": r64["kernel_ms"]}
        if "grad_fp64" in out:
            rec["res64"]["speedup_vs_fp64"] = (out["grad_fp64"]["ms_per_step"] /
                                               r64["ms_per_step"])
    rec.update(bench_extras(args, R, plan, obs, sky, D32, W32, modes, g["ms_per_step"]))
    if "chi2_mixed" in out and "chi2_fp64" in out:
        rec["chi2_only"] = {
            "mixed_terms_per_s": out["chi2_mixed"]["terms_per_s"],
            "fp64_terms_per_s": out["chi2_fp64"]["terms_per_s"],
            "mixed_ms": out["chi2_mixed"]["ms_per_step"],
            "fp64_ms": out["chi2_fp64"]["ms_per_step"]}
    plan.close()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        rec["cpu_baseline"] = cpu_baseline(problem_sample(name))
    return rec


def bench_extras(args, R, plan, obs, sky, D32, W32, modes, base_ms):
    """Float32-mixed chi^2 + gradient of the same workload with the rows
    beyond the static sky: per-call terms (a 2x2 G per timestep, antenna and
    channel, and Stokes per timestep, both with their gradients), the
    Gaussians replaced by exponential disks, and the out-of-core path with
    the data in pinned host memory (PCIe-inclusive; never the headline)."""
    import torch

    from rime_synth import Sky, random_die, rngs, stokes_per_time
    out = {}
    terms = obs.ntime * obs.nbl * obs.nchan * sky.nsrc
    dsky = R.DeviceSky.from_host(sky)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")

    def record(ms, **kw):
        r = {"ms_per_step": ms, "terms_per_s": terms / (ms * 1e-3),
             "vs_static_sky": ms / base_ms}
        r.update(kw)
        return r

    if "grad_terms" in modes:
        log("timing grad_terms")
        rng = rngs(1501)[0]
        die = torch.as_tensor(random_die(obs.ntime, obs.na, obs.nchan, rng), device="cuda")
        st = torch.as_tensor(stokes_per_time(sky, obs.ntime, rng), device="cuda")
        gdie, gst = torch.empty_like(die), torch.empty_like(st)
        ws = torch.empty(R.rime_workspace_size_ex(plan, R.MODE_CHI2_GRAD, R.MIXED, sky.nsrc,
                                                  die=True, grad_die=True, stokes_t=True,
                                                  grad_stokes_t=True),
                         dtype=torch.uint8, device="cuda")
        ms = timed(lambda: R.rime_chi2_ex(plan, dsky, R.MIXED, D32, W32, chi2, grad, ws,
                                          die=die, grad_die=gdie, stokes_t=st,
                                          grad_stokes_t=gst), args.steps, 1)[0]
        out["terms"] = record(ms, what="2x2 G per (timestep, antenna, channel) and Stokes per "
                                       "(timestep, source), with d chi2/dG and d chi2/dStokes_t; "
                                       "point sources on the matrix cores as in the plain call")
        log("grad_terms", out["terms"])
        del ws, die, st, gdie, gst
    if "grad_disk" in modes:
        log("timing grad_disk")
        disky = R.DeviceSky.from_host(Sky(lm=sky.lm, stokes=sky.stokes, alpha=sky.alpha,
                                          xshape=sky.gshape))
        ws = R.workspace(plan, R.MODE_CHI2_GRAD, R.MIXED, 1, sky.nsrc)
        ms = timed(lambda: R.rime_chi2_grad(plan, disky, R.MIXED, D32, W32, chi2, grad, ws),
                   args.steps, 1)[0]
        out["disk"] = record(ms, what=f"the {sky.ngsrc} Gaussians replaced by exponential disks")
        log("grad_disk", out["disk"])
        del ws
    if "grad_streamed" in modes:
        log("timing grad_streamed")
        # five chunks: at c2 each gives the per-baseline kernel whole rounds
        # of the device (1280 workgroups of 1024 threads)
        chunk_t = max(1, obs.ntime // 5)
        Dh, Wh = D32.cpu().pin_memory(), W32.cpu().pin_memory()
        ws = torch.empty(R.rime_streamed_workspace_size(plan, R.MODE_CHI2_GRAD, R.MIXED,
                                                        sky.nsrc, chunk_t),
                         dtype=torch.uint8, device="cuda")
        ms = timed(lambda: R.rime_chi2_streamed(plan, dsky, R.MIXED, Dh, Wh, chi2, grad,
                                                chunk_t, ws), args.steps, 1)[0]
        nbytes = Dh.numel() * Dh.element_size() + Wh.numel() * Wh.element_size()
        # the same bytes as two plain host-to-device copies: the PCIe floor
        dD, dW = torch.empty_like(D32), torch.empty_like(W32)
        h2d_ms = timed(lambda: (dD.copy_(Dh, non_blocking=True),
                                dW.copy_(Wh, non_blocking=True)), args.steps, 1)[0]
        del dD, dW
        out["streamed"] = record(ms, chunk_t=chunk_t, host_bytes=nbytes,
                                 host_bytes_per_s=nbytes / (ms * 1e-3),
                                 h2d_copy_ms=h2d_ms,
                                 what="data and weights in pinned host memory, uploaded in "
                                      f"chunks of {chunk_t} timesteps overlapping the compute "
                                      "(PCIe-inclusive); h2d_copy_ms: the same bytes as plain "
                                      "host-to-device copies")
        log("grad_streamed", out["streamed"])
        del ws, Dh, Wh
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------- #
# c3: batched proposals
# --------------------------------------------------------------------------- #

def bench_batch(args):
    import torch

    import paper_1501_07719_amd as R
    from rime_synth import make_batch_problem

    t_gen = time.perf_counter()
    pb = make_batch_problem()
    obs = pb.obs
    nset = len(pb.skies)
    nsrc = np.array([s.nsrc for s in pb.skies])
    npsrc = np.array([s.npsrc for s in pb.skies])
    log(f"generated c3: {nset} sets, {nsrc.sum()} sources (mean {nsrc.mean():.0f}) in "
        f"{time.perf_counter() - t_gen:.1f}s")
    plan = R.Plan(obs)
    D64, W64, D32, W32 = upload_data(R, plan, pb.truth, pb.noise, pb.weight)
    skies = [R.DeviceSky.from_host(s) for s in pb.skies]
    batch = R.Batch(plan, skies)
    per_vis = obs.ntime * obs.nbl * obs.nchan
    terms = per_vis * int(nsrc.sum())
    tp = per_vis * int(npsrc.sum())
    tg = terms - tp
    chi2 = torch.empty(nset, dtype=torch.float64, device="cuda")
    grad = torch.empty((batch.total_src, 10), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def batched(prec, graph):
        D, W = (D64, W64) if prec == R.FP64 else (D32, W32)
        ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, prec), dtype=torch.uint8,
                         device="cuda")

        def call():
            R.rime_chi2_batched(batch, prec, D, W, chi2, grad, ws, stream=stream,
                                use_graph=graph)
        return call, ws

    res = {}
    # default variant, one graph launch for all sets
    v_default = R.rime_batch_get_variant(batch, R.MODE_CHI2_GRAD, R.MIXED)
    call, ws = batched(R.MIXED, True)
    res["graph_default"] = timed(call, args.steps, 1)[0]
    log("graph default", R.rime_variant_info(R.MODE_CHI2_GRAD, R.MIXED, v_default),
        res["graph_default"])
    if not args.no_autotune:
        R.rime_batch_autotune(batch, R.MODE_CHI2_GRAD, R.MIXED, D32, W32, ws)
    v_tuned = R.rime_batch_get_variant(batch, R.MODE_CHI2_GRAD, R.MIXED)
    variant = R.rime_variant_info(R.MODE_CHI2_GRAD, R.MIXED, v_tuned)
    call, ws = batched(R.MIXED, True)
    res["graph_tuned"], _, tuned_steps = timed(call, args.steps, 1, per_step=True)
    log("graph tuned", variant, res["graph_tuned"])
    # the same launches without the graph, with the main kernel timed alone
    call, ws = batched(R.MIXED, False)
    res["stream_tuned"], (kms,), _ = timed(call, args.steps, 1, (plan.set_timing_events,))
    log("stream tuned", res["stream_tuned"], "kernel", kms)
    del ws, call
    # per-set loop: one rime_chi2_grad call per proposal, same variant
    plan.set_variant(R.MODE_CHI2_GRAD, R.MIXED, v_tuned)
    wsl = R.workspace(plan, R.MODE_CHI2_GRAD, R.MIXED, 1, int(nsrc.max()))
    offs = np.concatenate([[0], np.cumsum(nsrc)[:-1]])
    grads = [grad[int(o):int(o) + int(n)] for o, n in zip(offs, nsrc)]

    def loop():
        for i in range(nset):
            R.rime_chi2_grad(plan, skies[i], R.MIXED, D32, W32, chi2[i:i + 1], grads[i], wsl)
    res["loop_tuned"] = timed(loop, args.steps, 1)[0]
    log("per-set loop", res["loop_tuned"])
    # kernel times per set from the same loop, with HIP events around all
    # compute kernels of each call and around its per-baseline kernel: the
    # per-set pipelines of the batched call run these same kernels
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nset)]
    for e4 in ev:
        for e in e4:
            e.record()
    torch.cuda.synchronize()
    for i in range(nset):
        plan.set_timing_events(ev[i][0], ev[i][1])
        plan.set_main_events(ev[i][2], ev[i][3])
        R.rime_chi2_grad(plan, skies[i], R.MIXED, D32, W32, chi2[i:i + 1], grads[i], wsl)
    plan.set_timing_events(None, None)
    plan.set_main_events(None, None)
    torch.cuda.synchronize()
    set_kernel_ms = sum(e4[0].elapsed_time(e4[1]) for e4 in ev)
    set_main_ms = sum(e4[2].elapsed_time(e4[3]) for e4 in ev)
    log("per-set kernels", set_kernel_ms, "per-baseline kernels", set_main_ms)
    del wsl, ev
    if not args.no_fp64:
        call, ws = batched(R.FP64, True)
        res["graph_fp64"] = timed(call, max(1, args.steps // 2), 1)[0]
        log("graph fp64", res["graph_fp64"])
        del ws, call

    ms = res["graph_tuned"]
    rec = base_record(
        args, "source x visibility terms/s (chi2+grad, FP32-mixed), 1 GPU", terms / (ms * 1e-3),
        ms, "f32",
        f"c3: {nset} batched proposals of {nsrc.min()}..{nsrc.max()} sources "
        f"(sum {nsrc.sum()}, 30 % Gaussian) over {obs.na} antennas ({obs.nbl} baselines), "
        f"{obs.ntime} timesteps, {obs.nchan} channels, beam; one hipGraph launch",
        {"terms_per_eval": terms, "sets": nset})
    rec["evals_per_s"] = nset * 1e3 / ms
    rec["step_ms"] = step_stats(tuned_steps)
    mc = R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, R.MIXED, v_tuned)
    rec["config"]["precision"] = MIXED_PRECISION_MC if mc else MIXED_PRECISION
    if mc:
        # the matrix-core variant runs the per-set pipeline: the per-baseline
        # kernel for the Gaussian sources, the matrix cores for the points;
        # their times are the sums over the sets' calls in the per-set loop
        g = {"matrix_cores": True, "main_ms": set_main_ms, "kernel_ms": set_kernel_ms,
             "variant": variant}
        rec.update(rooflines(g, tp, tg, obs, None, None, npoint=npsrc))
        for k in ("roofline", "roofline_other"):
            rec[k]["kernel"] += ", summed over the 256 sets (per-set calls)"
    else:
        rec["roofline"] = roofline(alg_flops(tp, tg), kms, variant, None)
    rec["batched"] = {
        "graph_tuned_ms": ms, "graph_default_ms": res["graph_default"],
        "stream_tuned_ms": res["stream_tuned"], "per_set_loop_ms": res["loop_tuned"],
        "default_variant": R.rime_variant_info(R.MODE_CHI2_GRAD, R.MIXED, v_default),
        "default_matrix_cores": R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, R.MIXED, v_default),
        "tuned_variant": variant, "tuned_matrix_cores": mc,
        "speedup_graph_vs_loop": res["loop_tuned"] / ms,
        "speedup_tuned_vs_default": res["graph_default"] / ms}
    if "graph_fp64" in res:
        rec["fp64"] = {"ms_per_step": res["graph_fp64"],
                       "terms_per_s": terms / (res["graph_fp64"] * 1e-3),
                       "evals_per_s": nset * 1e3 / res["graph_fp64"]}
        rec["speedup_mixed_vs_fp64"] = res["graph_fp64"] / ms
    batch.close()
    plan.close()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        mid = int(np.argsort(nsrc)[nset // 2])
        rec["cpu_baseline"] = cpu_baseline(batch_sample(pb, mid))
    return rec


# --------------------------------------------------------------------------- #
# c0: latency of one small FP64 evaluation
# --------------------------------------------------------------------------- #

def bench_latency(args):
    import torch

    import paper_1501_07719_amd as R
    from rime_synth import make_problem

    pr = make_problem("c0")
    obs, sky = pr.obs, pr.sky
    plan = R.Plan(obs)
    D64, W64, _, _ = upload_data(R, plan, pr.truth, pr.noise, pr.weight)
    dsky = R.DeviceSky.from_host(sky)
    batch = R.Batch(plan, [dsky])
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
    ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, R.FP64), dtype=torch.uint8,
                     device="cuda")
    stream = torch.cuda.current_stream()
    terms = obs.ntime * obs.nbl * obs.nchan * sky.nsrc

    def graph_call():
        R.rime_chi2_batched(batch, R.FP64, D64, W64, chi2, grad, ws, stream=stream,
                            use_graph=True)

    def plain_call():
        R.rime_chi2_grad(plan, dsky, R.FP64, D64, W64, chi2, grad, ws)

    ms_graph, _, graph_steps = timed(graph_call, args.steps, args.warmup, per_step=True)
    ms_plain, (kms,), _ = timed(plain_call, args.steps, args.warmup, (plan.set_timing_events,))
    variant = R.rime_variant_info(R.MODE_CHI2_GRAD, R.FP64,
                                  plan.get_variant(R.MODE_CHI2_GRAD, R.FP64))
    rec = base_record(
        args, "source x visibility terms/s (chi2+grad, FP64), 1 GPU", terms / (ms_graph * 1e-3),
        ms_graph, "f64",
        f"c0: RIME chi2+grad, {obs.na} antennas ({obs.nbl} baselines), {obs.ntime} timesteps, "
        f"{obs.nchan} channels, {sky.npsrc} point sources, no beam; one hipGraph launch",
        {"terms_per_eval": terms, "precision": "fp64"})
    rec["evals_per_s"] = 1e3 / ms_graph
    rec["step_ms"] = step_stats(graph_steps)
    rec["latency_us"] = {"graph": ms_graph * 1e3, "stream": ms_plain * 1e3,
                         "main_kernel": kms * 1e3}
    flops = alg_flops(terms, 0)
    achieved = flops / (kms * 1e-3) / 1e12
    rec["roofline"] = {"bound": "latency", "achieved": achieved, "peak": PEAK_TFLOPS["f64"],
                       "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f64"],
                       "traffic": None,
                       "kernel": "rime_main<double, %d, %d, %d, chi2+grad>" % tuple(variant),
                       "kernel_ms": kms, "flops_per_launch": flops}
    batch.close()
    plan.close()
    if not args.no_cpu_baseline:
        import oracle.rime_oracle as O
        D = O.model_vis(obs, pr.truth) + pr.noise
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 10.0:
            O.chi2_and_grad(obs, sky, D, pr.weight)
            n += 1
        dt = (time.perf_counter() - t0) / n
        rec["cpu_baseline"] = {"value": terms / dt, "unit": "terms/s",
                               "cores": torch.get_num_threads(), "kind": "oracle",
                               "sample": f"the whole c0 workload, {n} evaluations, "
                                         f"{dt * 1e3:.1f} ms each"}
    return rec


def bench_points(args):
    """The c4 point-source comparison: the 1500 point sources of c4 (beam-free,
    and with the beam for chi^2) through every float32-mixed variant; the best
    per-baseline (VALU) variant against the best matrix-core variant."""
    import torch

    import paper_1501_07719_amd as R
    from rime_synth import Observation, make_problem

    pr = make_problem("c4", dense=False)
    pts = pr.sky.subset(pr.sky.npsrc, 0)
    obs_beam = pr.obs
    obs_free = Observation(**{**pr.obs.__dict__, "beam": False, "pointing": None, "gains": None})
    del pr
    shp = (obs_free.ntime, obs_free.nbl, obs_free.nchan, 4)
    g = torch.Generator(device="cuda")
    g.manual_seed(1501)
    nz = torch.randn(shp + (2,), dtype=torch.float32, device="cuda", generator=g) * 0.01
    D = torch.view_as_complex(nz)
    W = torch.full(shp, 1e4, dtype=torch.float32, device="cuda")
    del nz
    dsky = R.DeviceSky.from_host(pts)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((pts.nsrc, 10), dtype=torch.float64, device="cuda")
    terms = obs_free.ntime * obs_free.nbl * obs_free.nchan * pts.nsrc

    def compare(obs, mode):
        plan = R.Plan(obs)
        ws = R.workspace(plan, mode, R.MIXED, 1, pts.nsrc)
        res = {"valu": (None, None), "mfma": (None, None)}
        for vi in range(R.rime_variant_count(mode, R.MIXED)):
            plan.set_variant(mode, R.MIXED, vi)
            if mode == R.MODE_CHI2_GRAD:
                call = lambda: R.rime_chi2_grad(plan, dsky, R.MIXED, D, W, chi2, grad, ws)
            else:
                call = lambda: R.rime_chi2(plan, dsky, R.MIXED, D, W, chi2, ws)
            ms, _, _ = timed(call, args.steps, args.warmup)
            kind = "mfma" if R.rime_variant_matrix_cores(mode, R.MIXED, vi) else "valu"
            log(f"c4p beam={obs.beam} mode={mode} variant {vi} ({kind}): {ms:.2f} ms")
            if res[kind][0] is None or ms < res[kind][0]:
                res[kind] = (ms, list(R.rime_variant_info(mode, R.MIXED, vi)))
        plan.close()
        del ws
        torch.cuda.empty_cache()
        return {"valu_ms": res["valu"][0], "valu_variant": res["valu"][1],
                "mfma_ms": res["mfma"][0], "mfma_variant": res["mfma"][1],
                "speedup": res["valu"][0] / res["mfma"][0]}

    cmp = {"chi2_beam_free": compare(obs_free, R.MODE_CHI2),
           "chi2_with_beam": compare(obs_beam, R.MODE_CHI2),
           "chi2_grad_beam_free": compare(obs_free, R.MODE_CHI2_GRAD)}
    best = cmp["chi2_grad_beam_free"]["mfma_ms"]
    rec = base_record(
        args, "source x visibility terms/s (chi2+grad, FP32-mixed), 1 GPU", terms / (best * 1e-3),
        best, "f32",
        f"c4p: point subset of c4, {obs_free.na} antennas ({obs_free.nbl} baselines), "
        f"{obs_free.ntime} timesteps, {obs_free.nchan} channels, {pts.nsrc} point sources, "
        "beam-free; matrix-core variant against the per-baseline variants",
        {"terms_per_eval": terms, "precision": MIXED_PRECISION_MC})
    # the method's flops on the point terms, and beside them what the matrix
    # cores execute for them (as in the c2 line's roofline_other)
    flops = alg_flops(terms, 0)
    fl_exec = mfma_flops(obs_free, pts.nsrc)
    achieved = flops / (best * 1e-3) / 1e12
    rec["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f16_mfma"],
                       "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f16_mfma"],
                       "traffic": None,
                       "kernel": "all kernels of the call (point sources on the matrix cores)",
                       "kernel_ms": best, "flops_per_launch": flops,
                       "executed_mfma_flops_per_launch": fl_exec,
                       "executed_tflops": fl_exec / (best * 1e-3) / 1e12}
    rec["comparison"] = cmp
    return rec


def write_traffic(pairs, out_path, workload="c2"):
    """HBM bytes per launch of the chi^2 + gradient per-baseline kernel of
    `workload`, from FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by
    what the same counters read for the 1 GiB calibration copy; one entry per
    (FETCH_SIZE, WRITE_SIZE) pair of counter files.  Entries of an existing
    summary taken on the same kernel sources are kept unless replaced (same
    variant and workload)."""
    import csv
    import re
    import statistics

    pat = re.compile(r"rime_main<float, (\d+), (\d+), (\d+), 2, false>")

    def read(path):
        rows = list(csv.DictReader(open(path)))
        kern, copy, red, names = [], [], [], set()
        mc = any("pme_" in r["Kernel_Name"] for r in rows)
        for r in rows:
            m = pat.search(r["Kernel_Name"])
            if m:
                kern.append(float(r["Counter_Value"]))
                names.add(m.groups())
            elif "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) == 131072:
                copy.append(float(r["Counter_Value"]))
            elif "reduce_kernel" in r["Kernel_Name"]:
                red.append(float(r["Counter_Value"]))
        if len(names) != 1 or not copy:
            raise SystemExit(f"{path}: expected one chi2+grad kernel variant and the 1 GiB copy")
        return (statistics.mean(kern), copy[0], max(red) if red else None,
                [int(x) for x in names.pop()] + [int(mc)])

    entries = []
    for fetch_csv, write_csv in pairs:
        fk, fc, fr, var = read(fetch_csv)
        wk, wc, _, var_w = read(write_csv)
        if var != var_w:
            raise SystemExit("the two passes ran different variants")
        fscale, wscale = 1048576.0 / fc, 1048576.0 / wc
        fb, wb = fk * 1024 * fscale, wk * 1024 * wscale
        e = {"kernel": "rime_main<float, %d, %d, %d, 2, false>" % tuple(var[:3]),
             "variant": var, "workload": workload, "fetch_kib_raw": fk,
             "write_kib_raw": wk, "fetch_scale": fscale, "write_scale": wscale,
             "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
             "grad_mixed_bytes_per_launch": fb + wb}
        if fr:
            # the read-only sum of the same 1 GiB: its factor beside the copy's
            e["fetch_scale_read_only"] = 1048576.0 / fr
        entries.append(e)
    digest = kernel_source_digest()
    try:
        with open(out_path) as f:
            old = json.load(f)
    except (OSError, ValueError):
        old = {}
    if old.get("kernel_source_sha256") == digest:
        new_keys = {(tuple(e["variant"]), e["workload"]) for e in entries}
        entries = [e for e in old.get("entries", [])
                   if (tuple(e["variant"]), e["workload"]) not in new_keys] + entries
    out = {"entries": entries, "kernel_source_sha256": digest}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic, args.traffic, args.config)
        return
    if args.config in ("c1", "c2", "c4") and "grad_mixed" not in args.modes.split(","):
        # the line's value, roofline and traffic are those of grad_mixed
        raise SystemExit("bench.py: --modes must include grad_mixed (the timed headline)")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    # all work on one non-default stream (default priority): hipGraph capture
    # needs a stream other than the null stream
    with torch.cuda.stream(torch.cuda.Stream()):
        if args.config == "c3":
            rec = bench_batch(args)
        elif args.config == "c0":
            rec = bench_latency(args)
        elif args.config == "c4p":
            rec = bench_points(args)
        else:
            rec = bench_single(args)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
