"""Oracle parity of chi^2 and its gradient at full array geometry with every
source: one timestep of the c2 workload (64 antennas, all 2016 baselines,
1000 point + 500 Gaussian sources, 64 channels over 0.9-1.7 GHz, beam and
gains) and of the c4 workload (197 antennas, all 19306 baselines, 1500 point +
500 Gaussian sources, the first 4 of its 256 channels).

The observed data are the oracle's model of the perturbed truth sky plus
noise, rounded once to complex64 so that every precision and the oracle
consume the same values.  Checked per precision and kernel variant (the
default one, which puts the point sources on the matrix cores in the mixed
precisions, and the per-baseline one): chi^2 relative, the gradient per
parameter type (2-norm) and per component against the type's root mean
square, at 1e-12 for FP64 and 1e-5 for the mixed precisions; FP64 also per
component against 1e-3 of the type's largest entry.
"""
import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import make_problem
from tests._helpers import TOL, grad_component_errors, grad_errors, rel, round_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")

GEOMS = {"c2": dict(ntime=1), "c4": dict(ntime=1, nchan=256)}
CHANS = {"c2": (0, 64), "c4": (0, 4)}
_REF = {}


def say(*a):
    print("[gpu-geom]", *a, flush=True)


def reference(name):
    if name not in _REF:
        pr = make_problem(name, **GEOMS[name])
        c0, c1 = CHANS[name]
        obs = pr.obs.chan_slice(c0, c1)
        noise = pr.noise[:, :, c0:c1]
        say(name, "oracle", f"nbl={obs.nbl} nchan={obs.nchan} nsrc={pr.sky.nsrc}")
        D = O.model_vis(obs, pr.truth) + noise
        D, W = round_inputs(D, pr.weight[:, :, c0:c1], 1)
        c, g = O.chi2_and_grad(obs, pr.sky, D, W)
        _REF[name] = (obs, pr.sky, D, W, c, g)
    return _REF[name]


def variants(prec):
    """The plan's default variant and the 256-thread per-baseline one."""
    per_bl = next(i for i in range(R.rime_variant_count(R.MODE_CHI2_GRAD, prec))
                  if not R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, prec, i)
                  and R.rime_variant_info(R.MODE_CHI2_GRAD, prec, i)[0] == 256)
    return [None, per_bl]


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_full_geometry_gradient(name, prec):
    obs, sky, D, W, c, g = reference(name)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    Dd = torch.as_tensor(D, dtype=cdt, device="cuda")
    Wd = torch.as_tensor(W, dtype=rdt, device="cuda")
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    tol = TOL[prec]
    fails = []
    for vi in variants(prec):
        if vi is not None:
            plan.set_variant(R.MODE_CHI2_GRAD, prec, vi)
        used = plan.get_variant(R.MODE_CHI2_GRAD, prec)
        chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
        grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
        ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
        R.rime_chi2_grad(plan, dsky, prec, Dd, Wd, chi2, grad, ws)
        gg = grad.cpu().numpy()
        del ws
        ec = rel(chi2.item(), c)
        ge = grad_errors(gg, g, sky.npsrc)
        gc = grad_component_errors(gg, g, sky.npsrc)
        wc = max(gc.values())
        gr = grad_component_errors(gg, g, sky.npsrc, floor="rms")
        say(name, prec, used, R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, prec, used),
            f"chi2 rel {ec:.2e}", "per type", {k: f"{v:.1e}" for k, v in ge.items()},
            "per component", {k: f"{v:.1e}" for k, v in gc.items()},
            "rms floor", {k: f"{v:.1e}" for k, v in gr.items()})
        if not (ec <= tol and max(ge.values()) <= tol and max(gr.values()) <= tol):
            fails.append((used, ec, ge, gr))
        if prec == R.FP64 and wc > tol:
            fails.append((used, "component", wc))
        assert np.all(gg[:sky.npsrc, 7:] == 0.0)
    plan.close()
    assert not fails, fails
