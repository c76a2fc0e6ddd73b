"""Parity of the matrix-core point-source engine (float32-mixed variants that
form the point-source sums as the antenna x antenna product per timestep and
channel) against the CPU oracle, through the C ABI: visibilities, chi^2 and
gradient to the mixed tolerance (1e-5 of F_nu, 1e-5 relative).

The observations span several 32-antenna blocks with a ragged last block (up to
three blocks, where the forward runs one tile per workgroup, and five and
seven, where it pairs two), baselines in arbitrary order with swapped antenna
pairs across blocks (the engine then takes the conjugate of the stored pair),
a duplicate baseline and an autocorrelation, with and without the beam. Two cases end the channel
blocks of the phase planes with a partial block: 16 + 3 channels for small
planes, and 4 + 3 for planes of 1 MiB and more.
"""
import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import Observation, Sky, make_problem
from tests._helpers import (TOL, grad_component_errors, grad_component_worst, grad_errors, rel,
                            round_inputs, vis_error)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")


def say(*a):
    print("[gpu-mc]", *a, flush=True)


def mc_variants(mode, prec=None):
    prec = R.MIXED if prec is None else prec
    return [i for i in range(R.rime_variant_count(mode, prec))
            if R.rime_variant_matrix_cores(mode, prec, i)]


def problem(kind):
    rng = np.random.default_rng(17)
    if kind == "three_blocks":
        pr = make_problem("c1", ntime=2, nchan=3, npsrc=45, ngsrc=12, na=70, key=31)
        obs, sky = pr.obs, pr.sky
    elif kind == "shuffled_swapped":
        pr = make_problem("c1", ntime=2, nchan=2, npsrc=40, ngsrc=6, na=40, key=32)
        obs, sky = pr.obs, pr.sky
        n = obs.nbl
        perm = rng.permutation(n)
        a1, a2 = obs.ant1[perm].copy(), obs.ant2[perm].copy()
        sw = rng.random(n) < 0.5
        a1[sw], a2[sw] = a2[sw], a1[sw].copy()
        a1 = np.concatenate([a1, a1[:1], [35]]).astype(np.int32)
        a2 = np.concatenate([a2, a2[:1], [35]]).astype(np.int32)
        obs = Observation(**{**obs.__dict__, "ant1": a1, "ant2": a2})
    elif kind == "five_blocks_swapped":
        # 150 antennas: five blocks (the last ragged), so that the forward
        # pairs the P blocks of each Q block, with a lone block left over
        # where a Q block has an odd number of pairs; 300 of the baselines,
        # shuffled, half of them swapped
        pr = make_problem("c1", ntime=2, nchan=3, npsrc=40, ngsrc=6, na=150, key=37)
        obs, sky = pr.obs, pr.sky
        keep = rng.choice(obs.nbl, 300, replace=False)
        a1, a2 = obs.ant1[keep].copy(), obs.ant2[keep].copy()
        sw = rng.random(a1.size) < 0.5
        a1[sw], a2[sw] = a2[sw], a1[sw].copy()
        obs = Observation(**{**obs.__dict__, "ant1": a1.astype(np.int32),
                             "ant2": a2.astype(np.int32)})
    elif kind == "points_no_beam":
        pr = make_problem("c4", ntime=1, nchan=3, npsrc=50, ngsrc=0, na=45, key=33)
        obs = Observation(**{**pr.obs.__dict__, "beam": False, "pointing": None,
                             "gains": None})
        sky = pr.sky
    elif kind == "gauss_only":
        pr = make_problem("c1", ntime=1, nchan=2, npsrc=0, ngsrc=10, na=34, key=34)
        obs, sky = pr.obs, pr.sky
    elif kind == "ragged_channel_blocks":
        # small phase planes are written in blocks of 16 channels: 16 + 3
        pr = make_problem("c1", ntime=2, nchan=19, npsrc=40, ngsrc=8, na=40, key=35)
        obs, sky = pr.obs, pr.sky
    elif kind == "wide_planes":
        # 1200 sources x 224 padded antennas: 1.08 MB planes, written in blocks
        # of 4 channels (7 channels: 4 + 3); 60 of the baselines keep the
        # oracle small (the plane size depends on the antennas only)
        pr = make_problem("c4", ntime=1, nchan=7, npsrc=1200, ngsrc=0, na=197, key=36,
                          dense=False)
        obs, sky = pr.obs, pr.sky
        keep = np.sort(rng.choice(obs.nbl, 60, replace=False))
        obs = Observation(**{**obs.__dict__, "ant1": obs.ant1[keep].copy(),
                             "ant2": obs.ant2[keep].copy()})
    else:
        raise ValueError(kind)
    nz = np.random.default_rng(3).normal(0, 0.01, (obs.ntime, obs.nbl, obs.nchan, 4, 2))
    truth = Sky.from_params(sky.params() * (1 + 0.01 * np.random.default_rng(4).standard_normal(
        (sky.nsrc, 10))), sky.ngsrc)
    D = O.model_vis(obs, truth) + nz[..., 0] + 1j * nz[..., 1]
    W = np.full(D.shape, 1e4)
    return obs, sky, D, W


KINDS = ["three_blocks", "shuffled_swapped", "five_blocks_swapped", "points_no_beam",
         "gauss_only", "ragged_channel_blocks", "wide_planes"]


@pytest.mark.parametrize("kind", KINDS)
def test_matrix_core_engine(kind):
    obs, sky, D, W = problem(kind)
    D, W = round_inputs(D, W, R.MIXED)
    V = O.model_vis(obs, sky)
    c, g = O.chi2_and_grad(obs, sky, D, W)
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    Dd = torch.as_tensor(D, dtype=torch.complex64, device="cuda")
    Wd = torch.as_tensor(W, dtype=torch.float32, device="cuda")
    shp = (obs.ntime, obs.nbl, obs.nchan, 4)
    tol = TOL[R.MIXED]
    for vi in mc_variants(R.MODE_PREDICT):
        plan.set_variant(R.MODE_PREDICT, R.MIXED, vi)
        vis = torch.empty(shp, dtype=torch.complex64, device="cuda")
        R.rime_predict(plan, dsky, R.MIXED, vis,
                       R.workspace(plan, R.MODE_PREDICT, R.MIXED, 1, sky.nsrc))
        ev = vis_error(vis.cpu().numpy().astype(np.complex128), V, sky, obs)
        say(kind, "predict", vi, f"|dV|/F = {ev:.2e}")
        assert ev <= tol
    for vi in mc_variants(R.MODE_CHI2):
        plan.set_variant(R.MODE_CHI2, R.MIXED, vi)
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        R.rime_chi2(plan, dsky, R.MIXED, Dd, Wd, chi2,
                    R.workspace(plan, R.MODE_CHI2, R.MIXED, 1, sky.nsrc))
        e = rel(chi2.item(), c)
        say(kind, "chi2", vi, f"rel {e:.2e}")
        assert e <= tol
    for prec in (R.MIXED, R.MIXED_RES64):
        for vi in mc_variants(R.MODE_CHI2_GRAD, prec):
            plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
            chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
            grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
            R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad,
                             R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc))
            gg = grad.cpu().numpy()
            ge = grad_errors(gg, g, sky.npsrc)
            wc = max(grad_component_errors(gg, g, sky.npsrc, floor="rms").values())
            say(kind, "grad", prec, vi, f"chi2 rel {rel(chi2.item(), c):.2e}",
                {k: f"{v:.1e}" for k, v in ge.items()}, f"worst component (rms floor) {wc:.1e}",
                f"(1e-3 max floor {grad_component_worst(gg, g, sky.npsrc):.1e})")
            assert rel(chi2.item(), c) <= tol
            assert max(ge.values()) <= tol
            assert wc <= tol
    plan.close()


def test_batched_matrix_cores():
    """Batched proposals with a matrix-core variant (the single-sky pipeline
    once per set, in one launch sequence): equal to single calls of the same
    variant, graph replay equal to the eager call, two sets against the
    oracle to the mixed tolerance."""
    from rime_synth import make_batch_problem
    bp = make_batch_problem(nset=5, ntime=2, nchan=4, nmin=3, nmax=60, key=45)
    obs = bp.obs
    Dm = O.model_vis(obs, bp.truth.subset(50, 20)) + bp.noise
    D, W = round_inputs(Dm, bp.weight, R.MIXED)
    Dd = torch.as_tensor(D, dtype=torch.complex64, device="cuda")
    Wd = torch.as_tensor(W, dtype=torch.float32, device="cuda")
    plan = R.Plan(obs)
    skies = [R.DeviceSky.from_host(s) for s in bp.skies]
    batch = R.rime_batch_create(plan, skies)
    vi = mc_variants(R.MODE_CHI2_GRAD)[0]
    R.rime_batch_set_variant(batch, R.MODE_CHI2_GRAD, R.MIXED, vi)
    plan.set_variant(R.MODE_CHI2_GRAD, R.MIXED, vi)
    nset = len(skies)
    stream = torch.cuda.Stream()
    chi2 = torch.empty(nset, dtype=torch.float64, device="cuda")
    grad = torch.empty((batch.total_src, 10), dtype=torch.float64, device="cuda")
    ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, R.MIXED), dtype=torch.uint8,
                     device="cuda")
    say("batched", [s.nsrc for s in skies])
    with torch.cuda.stream(stream):
        R.rime_chi2_batched(batch, R.MIXED, Dd, Wd, chi2, grad, ws, stream=stream,
                            use_graph=False)
    stream.synchronize()
    cb, gb = chi2.cpu().numpy().copy(), grad.cpu().numpy().copy()
    for rep in range(3):
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work in between
        with torch.cuda.stream(stream):
            R.rime_chi2_batched(batch, R.MIXED, Dd, Wd, chi2, grad, ws, stream=stream,
                                use_graph=True)
        stream.synchronize()
        np.testing.assert_array_equal(cb, chi2.cpu().numpy())
        np.testing.assert_array_equal(gb, grad.cpu().numpy())
    off = 0
    c1 = torch.empty(1, dtype=torch.float64, device="cuda")
    for i, s in enumerate(skies):
        g1 = torch.empty((s.nsrc, 10), dtype=torch.float64, device="cuda")
        R.rime_chi2_grad(plan, s, R.MIXED, Dd, Wd, c1, g1,
                         R.workspace(plan, R.MODE_CHI2_GRAD, R.MIXED, 1, s.nsrc))
        assert rel(cb[i], c1.item()) <= 1e-12
        ge = grad_errors(gb[off:off + s.nsrc], g1.cpu().numpy(), s.npsrc)
        assert max(ge.values()) <= 1e-12, (i, ge)
        off += s.nsrc
    off = 0
    for i, s in enumerate(bp.skies[:2]):
        c, g = O.chi2_and_grad(obs, s, D, W)
        assert rel(cb[i], c) <= TOL[R.MIXED]
        ge = grad_errors(gb[off:off + s.nsrc], g, s.npsrc)
        say("batched vs oracle", i, f"chi2 {rel(cb[i], c):.1e}",
            {k: f"{v:.1e}" for k, v in ge.items()})
        assert max(ge.values()) <= TOL[R.MIXED], ge
        off += s.nsrc
    batch.close()
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_bitwise_deterministic(prec):
    """Fixed-order reductions: repeated chi^2 + gradient calls (the default
    variant: matrix cores in float32-mixed) give bitwise identical results."""
    obs, sky, D, W = problem("three_blocks")
    D, W = round_inputs(D, W, prec)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    Dd = torch.as_tensor(D, dtype=cdt, device="cuda")
    Wd = torch.as_tensor(W, dtype=rdt, device="cuda")
    ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
    res = []
    for rep in range(3):
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        ws.fill_(rep)  # stale workspace contents must not matter
        R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad, ws)
        res.append((chi2.cpu().numpy(), grad.cpu().numpy()))
    for c, g in res[1:]:
        np.testing.assert_array_equal(c, res[0][0])
        np.testing.assert_array_equal(g, res[0][1])
    plan.close()


def test_high_dynamic_range():
    """A sky spanning 1e5 in brightness (I from 10 Jy down to 1e-4 Jy) with
    Q = U = V = 0 on a third of the sources: the faint sources sit far below
    the power-of-two operand scale that the brightest source sets for the
    fp16 hi/lo products.  Matrix-core variants of both mixed precisions
    against the oracle: visibilities, chi^2, and the gradient per type and per
    component (against the type's root mean square), for all sources and for
    the faint ones (I < 1e-3 Jy) on their own scale."""
    pr = make_problem("c1", ntime=2, nchan=3, npsrc=60, ngsrc=10, na=40, key=38)
    obs, sky = pr.obs, pr.sky
    rng = np.random.default_rng(38)
    st = sky.stokes.copy()
    I = 10.0 * 10.0 ** (-5.0 * rng.random(sky.nsrc))
    I[0], I[1] = 10.0, 1e-4
    frac = st[:, 1:4] / st[:, :1]
    st[:, 0] = I
    st[:, 1:4] = I[:, None] * frac
    st[::3, 1:4] = 0.0
    sky = Sky(lm=sky.lm, stokes=st, alpha=sky.alpha, gshape=sky.gshape)
    truth = Sky.from_params(sky.params() * (1 + 0.01 * rng.standard_normal((sky.nsrc, 10))),
                            sky.ngsrc)
    nz = rng.normal(0, 0.01, (obs.ntime, obs.nbl, obs.nchan, 4, 2))
    D = O.model_vis(obs, truth) + nz[..., 0] + 1j * nz[..., 1]
    D, W = round_inputs(D, np.full(D.shape, 1e4), R.MIXED)
    V = O.model_vis(obs, sky)
    c, g = O.chi2_and_grad(obs, sky, D, W)
    faint = np.flatnonzero(I < 1e-3)
    assert faint.size >= 5
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    Dd = torch.as_tensor(D, dtype=torch.complex64, device="cuda")
    Wd = torch.as_tensor(W, dtype=torch.float32, device="cuda")
    tol = TOL[R.MIXED]
    for vi in mc_variants(R.MODE_PREDICT):
        plan.set_variant(R.MODE_PREDICT, R.MIXED, vi)
        vis = torch.empty((obs.ntime, obs.nbl, obs.nchan, 4), dtype=torch.complex64,
                          device="cuda")
        R.rime_predict(plan, dsky, R.MIXED, vis,
                       R.workspace(plan, R.MODE_PREDICT, R.MIXED, 1, sky.nsrc))
        ev = vis_error(vis.cpu().numpy().astype(np.complex128), V, sky, obs)
        say("hdr predict", vi, f"|dV|/F = {ev:.2e}")
        assert ev <= tol
    for prec in (R.MIXED, R.MIXED_RES64):
        for vi in mc_variants(R.MODE_CHI2_GRAD, prec):
            plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
            chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
            grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
            R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad,
                             R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc))
            gg = grad.cpu().numpy()
            ge = grad_errors(gg, g, sky.npsrc)
            wc = max(grad_component_errors(gg, g, sky.npsrc, floor="rms").values())
            # faint sources on their own scale: per column (l .. alpha), the
            # floor is the root mean square of the faint-source components
            a, b = gg[faint, :7], g[faint, :7]
            floor = np.sqrt(np.mean(b * b, axis=0))
            wf = float((np.abs(a - b) / np.maximum(np.abs(b), floor)).max())
            say("hdr grad", prec, vi, f"chi2 rel {rel(chi2.item(), c):.2e}",
                {k: f"{v:.1e}" for k, v in ge.items()}, f"worst {wc:.1e} faint {wf:.1e}")
            assert rel(chi2.item(), c) <= tol
            assert max(ge.values()) <= tol
            assert wc <= tol and wf <= tol
    plan.close()
