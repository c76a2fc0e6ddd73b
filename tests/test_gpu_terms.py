"""Per-call terms of eq. 1 beyond the sky, against the oracle:
- the direction-independent 2x2 term G_p(t, nu), applied outside the source
  sum (V = G_p X G_q^H), with d chi^2 / dG;
- brightness per timestep (Table rime_input's ntime x nsrc brightness), with
  d chi^2 / d stokes_t;
- both together.
Every precision and every chi^2 + gradient kernel variant (per-baseline and
matrix-core), the gradient per type and per component against the type's
root mean square at the precision's bar, and the G and per-timestep
gradients in 2-norm and per entry against their root mean square."""
import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import Observation, make_problem, perturb, random_die, rngs, stokes_per_time
from tests._helpers import (TOL, grad_component_errors, grad_errors, rel, round_inputs,
                            vis_error)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")


def say(*a):
    print("[gpu-terms]", *a, flush=True)


def arr_errors(a, b):
    """(2-norm relative error, worst entry error against the root mean square)."""
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    nb = np.linalg.norm(b)
    rms = nb / np.sqrt(b.size)
    return float(np.linalg.norm(a - b) / nb), float((np.abs(a - b) / np.maximum(np.abs(b), rms)).max())


_REF = {}


def problem(kind):
    if kind not in _REF:
        pr = make_problem("c1", ntime=3, nchan=4, npsrc=34, ngsrc=8, na=40, key=95)
        # G carries the gains: the observation has none of its own
        obs = Observation(**{**pr.obs.__dict__, "gains": None})
        r = rngs(95)[5]
        sky = pr.sky
        die = random_die(obs.ntime, obs.na, obs.nchan, r) if kind in ("die", "both") else None
        st = stokes_per_time(sky, obs.ntime, r) if kind in ("stokes_t", "both") else None
        truth = perturb(sky, r)
        die_true = None if die is None else die * (1 + 0.01 * r.standard_normal(die.shape))
        st_true = None if st is None else st * (1 + 0.01 * r.standard_normal(st.shape))
        D = O.model_vis(obs, truth, die=die_true, stokes_t=st_true) + pr.noise
        D, W = round_inputs(D, pr.weight, 1)
        V = O.model_vis(obs, sky, die=die, stokes_t=st)
        ref = O.chi2_and_grad_ext(obs, sky, D, W, die=die, stokes_t=st)
        _REF[kind] = (obs, sky, die, st, D, W, V, ref)
    return _REF[kind]


def dev(x, dt):
    return None if x is None else torch.as_tensor(np.ascontiguousarray(x), dtype=dt,
                                                  device="cuda")


@pytest.mark.parametrize("kind", ["die", "stokes_t", "both"])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_terms_against_oracle(kind, prec):
    obs, sky, die, st, D, W, V, ref = problem(kind)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    Dd, Wd = dev(D, cdt), dev(W, rdt)
    die_d = dev(die, torch.complex128)
    st_d = dev(st, torch.float64)
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    tol = TOL[prec]
    if prec != R.MIXED_RES64:
        for vi in range(R.rime_variant_count(R.MODE_PREDICT, prec)):
            plan.set_variant(R.MODE_PREDICT, prec, vi)
            vis = torch.empty((obs.ntime, obs.nbl, obs.nchan, 4), dtype=cdt, device="cuda")
            ws = torch.empty(R.rime_workspace_size_ex(plan, R.MODE_PREDICT, prec, sky.nsrc,
                                                      die=die is not None,
                                                      stokes_t=st is not None),
                             dtype=torch.uint8, device="cuda")
            R.rime_predict_ex(plan, dsky, prec, vis, ws, die=die_d, stokes_t=st_d)
            ev = vis_error(vis.cpu().numpy().astype(np.complex128), V, sky, obs)
            say(kind, prec, "predict", vi, f"{ev:.1e}")
            assert ev <= tol
    for vi in range(R.rime_variant_count(R.MODE_CHI2_GRAD, prec)):
        plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
        ws = torch.empty(R.rime_workspace_size_ex(plan, R.MODE_CHI2_GRAD, prec, sky.nsrc,
                                                  die=die is not None,
                                                  grad_die=die is not None,
                                                  stokes_t=st is not None,
                                                  grad_stokes_t=st is not None),
                         dtype=torch.uint8, device="cuda")
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        gdie = None if die is None else torch.empty_like(die_d)
        gst = None if st is None else torch.empty_like(st_d)
        R.rime_chi2_ex(plan, dsky, prec, Dd, Wd, chi2, grad, ws, die=die_d, grad_die=gdie,
                       stokes_t=st_d, grad_stokes_t=gst)
        gg = grad.cpu().numpy()
        ge = grad_errors(gg, ref["grad"], sky.npsrc)
        gr = grad_component_errors(gg, ref["grad"], sky.npsrc, floor="rms")
        msg = [f"chi2 rel {rel(chi2.item(), ref['chi2']):.1e}",
               f"grad {max(ge.values()):.1e} / {max(gr.values()):.1e}"]
        assert rel(chi2.item(), ref["chi2"]) <= tol
        assert max(ge.values()) <= tol, ge
        assert max(gr.values()) <= tol, gr
        if die is not None:
            e2, ec = arr_errors(gdie.cpu().numpy(), ref["grad_die"])
            msg.append(f"dG {e2:.1e} / {ec:.1e}")
            assert e2 <= tol and ec <= tol
        if st is not None:
            e2, ec = arr_errors(gst.cpu().numpy(), ref["grad_stokes_t"])
            msg.append(f"dStokes_t {e2:.1e} / {ec:.1e}")
            assert e2 <= tol and ec <= tol
        say(kind, prec, "grad", vi, *msg)
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_identity_die_is_the_plain_call(prec):
    """G = I per (t, antenna, channel) gives the plain call's results."""
    obs, sky, _, _, D, W, _, _ = problem("die")
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    Dd, Wd = dev(D, cdt), dev(W, rdt)
    eye = np.broadcast_to(np.eye(2), (obs.ntime, obs.na, obs.nchan, 2, 2))
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    out = []
    for use_die in (False, True):
        ws = torch.empty(R.rime_workspace_size_ex(plan, R.MODE_CHI2_GRAD, prec, sky.nsrc,
                                                  die=True, grad_die=True),
                         dtype=torch.uint8, device="cuda")
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        if use_die:
            R.rime_chi2_ex(plan, dsky, prec, Dd, Wd, chi2, grad, ws,
                           die=dev(eye, torch.complex128))
        else:
            R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad, ws)
        out.append((chi2.item(), grad.cpu().numpy()))
    assert rel(out[1][0], out[0][0]) <= 1e-15
    ge = grad_errors(out[1][1], out[0][1], sky.npsrc)
    assert max(ge.values()) <= 1e-14, ge
    plan.close()


def test_terms_reject_bad_arguments():
    obs, sky, die, _, D, W, _, _ = problem("die")
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    Dd, Wd = dev(D, torch.complex128), dev(W, torch.float64)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty((obs.ntime, obs.na, obs.nchan, 2, 2), dtype=torch.complex128, device="cuda")
    ws = torch.empty(R.rime_workspace_size_ex(plan, R.MODE_CHI2, 0, sky.nsrc, die=True),
                     dtype=torch.uint8, device="cuda")
    # a G gradient without a source gradient (chi^2 only), and without G
    with pytest.raises(R.RimeError) as e:
        R.rime_chi2_ex(plan, dsky, R.FP64, Dd, Wd, chi2, None, ws, die=g, grad_die=g)
    assert e.value.status == 1
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(R.RimeError) as e:
        R.rime_chi2_ex(plan, dsky, R.FP64, Dd, Wd, chi2, grad, ws, grad_die=g)
    assert e.value.status == 1
    plan.close()
