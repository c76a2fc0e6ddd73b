"""A third source morphology, the elliptical exponential disk (a Sersic
profile of index 1: the paper's extension point of adding a source type with
its own loop), with its adjoint: parity against the oracle for skies that mix
points, Gaussians and disks, in every precision and every kernel variant,
plus the zero-size disk (a point source) and a batch with disks."""
import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import Sky, add_disks, make_problem, perturb, rngs
from tests._helpers import (TOL, grad_component_errors, grad_errors, rel, round_inputs,
                            vis_error)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")


def say(*a):
    print("[gpu-disk]", *a, flush=True)


_REF = {}


def problem(kind="mixed"):
    if kind not in _REF:
        pr = make_problem("c1", ntime=2, nchan=5, npsrc=30, ngsrc=10, na=24, key=81)
        r = rngs(81)[5]
        sky = add_disks(pr.sky, 12, r)
        if kind == "zero_size":
            sky = Sky(lm=sky.lm, stokes=sky.stokes, alpha=sky.alpha, gshape=sky.gshape,
                      xshape=np.concatenate([np.zeros((12, 2)), sky.xshape[:, 2:]], axis=1))
        truth = perturb(sky, r)
        D = O.model_vis(pr.obs, truth) + pr.noise
        D, W = round_inputs(D, pr.weight, 1)
        V = O.model_vis(pr.obs, sky)
        c, g = O.chi2_and_grad(pr.obs, sky, D, W)
        _REF[kind] = (pr.obs, sky, D, W, V, c, g)
    return _REF[kind]


def dev_data(D, W, prec):
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    return (torch.as_tensor(D, dtype=cdt, device="cuda"),
            torch.as_tensor(W, dtype=rdt, device="cuda"))


@pytest.mark.parametrize("kind", ["mixed", "zero_size"])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_disks_all_variants(kind, prec):
    obs, sky, D, W, V, c_ref, g_ref = problem(kind)
    Dd, Wd = dev_data(D, W, prec)
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    assert dsky.nxsrc == 12 and dsky.ngsrc == 10
    tol = TOL[prec]
    if prec != R.MIXED_RES64:
        for vi in range(R.rime_variant_count(R.MODE_PREDICT, prec)):
            plan.set_variant(R.MODE_PREDICT, prec, vi)
            vis = torch.empty((obs.ntime, obs.nbl, obs.nchan, 4),
                              dtype=torch.complex128 if prec == R.FP64 else torch.complex64,
                              device="cuda")
            R.rime_predict(plan, dsky, prec, vis,
                           R.workspace(plan, R.MODE_PREDICT, prec, 1, sky.nsrc))
            ev = vis_error(vis.cpu().numpy().astype(np.complex128), V, sky, obs)
            say(kind, prec, "predict", vi, f"{ev:.1e}")
            assert ev <= tol
    for vi in range(R.rime_variant_count(R.MODE_CHI2_GRAD, prec)):
        plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad,
                         R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc))
        gg = grad.cpu().numpy()
        ge = grad_errors(gg, g_ref, sky.npsrc)
        gr = grad_component_errors(gg, g_ref, sky.npsrc, floor="rms")
        say(kind, prec, "grad", vi, f"chi2 rel {rel(chi2.item(), c_ref):.1e}",
            {k: f"{v:.1e}" for k, v in ge.items()}, "rms floor",
            f"{max(gr.values()):.1e}")
        assert rel(chi2.item(), c_ref) <= tol
        assert max(ge.values()) <= tol, ge
        assert max(gr.values()) <= tol, gr
        # disk rows carry their shape gradient, point rows none
        assert np.all(gg[:sky.npsrc, 7:] == 0.0)
        if kind == "mixed":
            assert np.all(np.abs(gg[sky.npsrc + sky.ngsrc:, 7:]) > 0.0)
    plan.close()


def test_zero_size_disk_is_a_point():
    """Disks of zero size reproduce the same sources as points (FP64)."""
    obs, sky, D, W, _, _, _ = problem("zero_size")
    n0 = sky.npsrc + sky.ngsrc
    as_points = Sky(lm=np.concatenate([sky.lm[n0:], sky.lm[:n0]]),
                    stokes=np.concatenate([sky.stokes[n0:], sky.stokes[:n0]]),
                    alpha=np.concatenate([sky.alpha[n0:], sky.alpha[:n0]]), gshape=sky.gshape)
    plan = R.Plan(obs)
    out = []
    for s in (sky, as_points):
        vis = torch.empty((obs.ntime, obs.nbl, obs.nchan, 4), dtype=torch.complex128,
                          device="cuda")
        R.rime_predict(plan, R.DeviceSky.from_host(s), R.FP64, vis,
                       R.workspace(plan, R.MODE_PREDICT, R.FP64, 1, s.nsrc))
        out.append(vis.cpu().numpy())
    F = O.total_flux(sky, obs.freq, obs.ref_freq).max()
    err = np.abs(out[0] - out[1]).max() / F
    say("zero size vs points", f"{err:.1e}")
    assert err <= 1e-14
    plan.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batched_with_disks(prec):
    """Batched sets with disks equal single calls of the same variant."""
    obs, sky, D, W, _, _, _ = problem("mixed")
    Dd, Wd = dev_data(D, W, prec)
    plan = R.Plan(obs)
    skies = [R.DeviceSky.from_host(sky),
             R.DeviceSky.from_host(sky.subset(10, 4, 6)),
             R.DeviceSky.from_host(sky.subset(0, 0, 12))]
    batch = R.rime_batch_create(plan, skies)
    vi = next(i for i in range(R.rime_variant_count(R.MODE_CHI2_GRAD, prec))
              if not R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, prec, i)
              and R.rime_variant_info(R.MODE_CHI2_GRAD, prec, i)[0] == 256)
    R.rime_batch_set_variant(batch, R.MODE_CHI2_GRAD, prec, vi)
    plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
    chi2 = torch.empty(len(skies), dtype=torch.float64, device="cuda")
    grad = torch.empty((batch.total_src, 10), dtype=torch.float64, device="cuda")
    ws = torch.empty(batch.workspace_size(R.MODE_CHI2_GRAD, prec), dtype=torch.uint8,
                     device="cuda")
    R.rime_chi2_batched(batch, prec, Dd, Wd, chi2, grad, ws)
    cb, gb = chi2.cpu().numpy(), grad.cpu().numpy()
    off = 0
    c1 = torch.empty(1, dtype=torch.float64, device="cuda")
    for i, s in enumerate(skies):
        g1 = torch.empty((s.nsrc, 10), dtype=torch.float64, device="cuda")
        R.rime_chi2_grad(plan, s, prec, Dd, Wd, c1, g1,
                         R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, s.nsrc))
        assert rel(cb[i], c1.item()) <= 1e-12
        ge = grad_errors(gb[off:off + s.nsrc], g1.cpu().numpy(), s.npsrc)
        say("batched", prec, i, {k: f"{v:.1e}" for k, v in ge.items()})
        assert max(ge.values()) <= 1e-10, (i, ge)
        off += s.nsrc
    batch.close()
    plan.close()
