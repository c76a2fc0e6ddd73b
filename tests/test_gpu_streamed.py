"""Out-of-core evaluation (the paper's subdivision along time, Section 4
"Scaling the RIME"): data and weights in pinned host memory, streamed to the
device in chunks of timesteps through two staging buffers.  chi^2 and its
gradient are additive over time, so the streamed result must equal the
in-memory one up to the grouping of the final sums (1e-12 relative in every
precision), and the oracle to the precision's parity bar, for chunk sizes
that divide the time axis, leave a ragged last chunk, take one timestep at a
time, or cover it in one chunk."""
import numpy as np
import pytest

import oracle.rime_oracle as O
from tests._helpers import TOL, grad_errors, rel, round_inputs, small_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")


def say(*a):
    print("[gpu-stream]", *a, flush=True)


_REF = {}


def problem(prec):
    key = "mixed" if prec != R.FP64 else "fp64"
    if key not in _REF:
        pr, D, W = small_problem("c1", ntime=5, nchan=4, npsrc=40, ngsrc=12, na=40, key=71)
        D, W = round_inputs(D, W, prec)
        c, g = O.chi2_and_grad(pr.obs, pr.sky, D, W)
        _REF[key] = (pr.obs, pr.sky, D, W, c, g)
    return _REF[key]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_streamed_matches_in_memory_and_oracle(prec):
    obs, sky, D, W, c_ref, g_ref = problem(prec)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    Dh = torch.as_tensor(D, dtype=cdt).pin_memory()
    Wh = torch.as_tensor(W, dtype=rdt).pin_memory()
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
    ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
    R.rime_chi2_grad(plan, dsky, prec, Dh.cuda(), Wh.cuda(), chi2, grad, ws)
    c_mem, g_mem = chi2.item(), grad.cpu().numpy()
    del ws
    for chunk_t in (1, 2, 3, 5, 9):
        for with_grad in (True, False):
            n = R.rime_streamed_workspace_size(
                plan, R.MODE_CHI2_GRAD if with_grad else R.MODE_CHI2, prec, sky.nsrc, chunk_t)
            ws = torch.empty(n, dtype=torch.uint8, device="cuda")
            c = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            g = torch.full((sky.nsrc, 10), np.nan, dtype=torch.float64, device="cuda")
            say(prec, chunk_t, with_grad, n)
            R.rime_chi2_streamed(plan, dsky, prec, Dh, Wh, c, g if with_grad else None, chunk_t,
                                 ws)
            assert R.rime_domain_status(ws) == 0
            cs = c.item()
            assert rel(cs, c_mem) <= 1e-12, (chunk_t, cs, c_mem)
            assert rel(cs, c_ref) <= TOL[prec]
            if with_grad:
                gs = g.cpu().numpy()
                e_mem = grad_errors(gs, g_mem, sky.npsrc)
                e_ref = grad_errors(gs, g_ref, sky.npsrc)
                say(prec, chunk_t, f"chi2 rel {rel(cs, c_ref):.1e}",
                    f"vs in-memory {max(e_mem.values()):.1e}", f"vs oracle {max(e_ref.values()):.1e}")
                assert max(e_mem.values()) <= 1e-12, e_mem
                assert max(e_ref.values()) <= TOL[prec], e_ref
    plan.close()


def test_streamed_rejects_bad_arguments():
    obs, sky, D, W, _, _ = problem(R.FP64)
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    Dh = torch.as_tensor(D).pin_memory()
    Wh = torch.as_tensor(W).pin_memory()
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RimeError) as e:
        R.rime_chi2_streamed(plan, dsky, R.FP64, Dh, Wh, chi2, None, 2, small)
    assert e.value.status == 2
    ws = torch.empty(R.rime_streamed_workspace_size(plan, R.MODE_CHI2, R.FP64, sky.nsrc, 2),
                     dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RimeError) as e:
        R.rime_chi2_streamed(plan, dsky, R.FP64, Dh, Wh, chi2, None, 0, ws)
    assert e.value.status == 1
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_streamed_from_pageable_memory(prec):
    """Data and weights in ordinary (pageable) host memory: the uploads lose
    their overlap but keep their order against the compute of the chunk that
    used the staging buffer before, so results equal the in-memory call to
    1e-12, with several chunks through each of the two staging buffers."""
    obs, sky, D, W, _, _ = problem(prec)
    cdt = torch.complex128 if prec == R.FP64 else torch.complex64
    rdt = torch.float64 if prec == R.FP64 else torch.float32
    Dh, Wh = torch.as_tensor(D, dtype=cdt).contiguous(), torch.as_tensor(W, dtype=rdt).contiguous()
    assert not Dh.is_pinned() and not Wh.is_pinned()
    plan = R.Plan(obs)
    dsky = R.DeviceSky.from_host(sky)
    chi2 = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((sky.nsrc, 10), dtype=torch.float64, device="cuda")
    ws = R.workspace(plan, R.MODE_CHI2_GRAD, prec, 1, sky.nsrc)
    R.rime_chi2_grad(plan, dsky, prec, Dh.cuda(), Wh.cuda(), chi2, grad, ws)
    c_mem, g_mem = chi2.item(), grad.cpu().numpy()
    wss = torch.empty(R.rime_streamed_workspace_size(plan, R.MODE_CHI2_GRAD, prec, sky.nsrc, 1),
                      dtype=torch.uint8, device="cuda")
    for rep in range(3):
        c = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        g = torch.full((sky.nsrc, 10), np.nan, dtype=torch.float64, device="cuda")
        R.rime_chi2_streamed(plan, dsky, prec, Dh, Wh, c, g, 1, wss)
        e = max(grad_errors(g.cpu().numpy(), g_mem, sky.npsrc).values())
        say("pageable", prec, rep, f"chi2 rel {rel(c.item(), c_mem):.1e} grad {e:.1e}")
        assert rel(c.item(), c_mem) <= 1e-12 and e <= 1e-12
    plan.close()
