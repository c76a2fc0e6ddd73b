"""The allocation-free entry point rime_chi2_grad_noalloc against
rime_chi2_grad with a caller-owned workspace: two calls in a row on one
device, the second with a smaller problem (the library's fixed block keeps
the first call's contents), each equal to the workspace call of the same
kernel variant to the parity bar (and, the kernels being the same, bitwise);
a problem whose workspace exceeds the fixed block is rejected before
anything is enqueued."""
import numpy as np
import pytest

from rime_synth import make_problem
from tests._helpers import TOL, grad_errors, rel, round_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")

import oracle.rime_oracle as O  # noqa: E402


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)


def _data(pr, prec):
    D = O.model_vis(pr.obs, pr.truth) + pr.noise
    D, W = round_inputs(D, pr.weight, prec)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    return (torch.as_tensor(D, dtype=cdt, device="cuda"),
            torch.as_tensor(W, dtype=rdt, device="cuda"))


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_matches_workspace_call(prec):
    problems = [make_problem("c0"),  # 7 antennas, 10 t, 16 ch, 20 sources
                make_problem("c1", ntime=2, nchan=3, npsrc=6, ngsrc=3, na=5, key=91)]
    for i, pr in enumerate(problems):
        plan = R.Plan(pr.obs)
        sky = R.DeviceSky.from_host(pr.sky)
        Dd, Wd = _data(pr, prec)
        out = []
        for noalloc in (True, False):
            chi2 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            grad = torch.full((sky.nsrc, 10), np.nan, dtype=torch.float64, device="cuda")
            if noalloc:
                R.rime_chi2_grad_noalloc(plan, sky, prec, Dd, Wd, chi2, grad)
            else:
                ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
                R.rime_chi2_grad(plan, sky, prec, Dd, Wd, chi2, grad, ws)
            torch.cuda.synchronize()
            out.append((chi2.item(), grad.cpu().numpy()))
        (c_na, g_na), (c_ws, g_ws) = out
        ge = grad_errors(g_na, g_ws, sky.npsrc)
        say(prec, i, f"chi2 {c_na:.6e} vs {c_ws:.6e}", {k: f"{v:.1e}" for k, v in ge.items()},
            "bitwise" if c_na == c_ws and np.array_equal(g_na, g_ws) else "differs")
        assert np.isfinite(c_na) and np.all(np.isfinite(g_na))
        assert rel(c_na, c_ws) <= TOL[prec]
        assert max(ge.values()) <= TOL[prec], ge
        plan.close()


def test_noalloc_rejects_oversized_problem():
    """The c2 observation with 1500 sources needs far more than the fixed
    32 MiB block: RIME_ERR_WORKSPACE, nothing enqueued, outputs untouched."""
    pr = make_problem("c1", ntime=4, nchan=16, dense=False)
    plan = R.Plan(pr.obs)
    sky = R.DeviceSky.from_host(pr.sky)
    assert plan.workspace_size(R.MODE_CHI2_GRAD, R.MIXED, 1, sky.nsrc) > 32 << 20
    shp = (pr.obs.ntime, pr.obs.nbl, pr.obs.nchan, 4)
    Dd = torch.zeros(shp, dtype=torch.complex64, device="cuda")
    Wd = torch.ones(shp, dtype=torch.float32, device="cuda")
    chi2 = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    grad = torch.full((sky.nsrc, 10), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RimeError) as e:
        R.rime_chi2_grad_noalloc(plan, sky, R.MIXED, Dd, Wd, chi2, grad)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert chi2.item() == -1.0 and bool((grad == -1.0).all())
    plan.close()
