"""Full-size checks of the HIP path, at the benchmark workloads and in the launch
configuration that the benchmark times (the library's autotuned variant for
the mixed path and, on the 64-antenna workload, for FP64 too).

At these sizes the oracle cannot evaluate the whole sum, so the checks are:
- Sampled parity: model visibilities of whole (timestep, channel) slices, all
  baselines and all sources, against the oracle one slice at a time.  The bar
  is the parity bar, |dV| <= tol * F_nu.
- chi^2 properties: the chi^2 of both chi^2 entry points equals
  sum w |V - D|^2, formed on the device from the FP64 model visibilities
  (FP64 to 1e-12, mixed to 1e-5).
- Gradient properties: the FP64 gradient against central differences of the
  FP64 chi^2 along random directions, one parameter type at a time, and the
  mixed gradient against the FP64 gradient (per type, 1e-5).

The data D = model(truth) + noise is formed on the device.  The oracle never
sees D: it only evaluates model visibilities of the generator's sky.
"""
import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import Sky, make_problem
from tests._helpers import TOL, grad_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1501_07719_amd")

NAMES = ["l", "m", "I", "Q", "U", "V", "alpha", "el", "em", "R"]


def say(*a):
    print("[gpu-full]", *a, flush=True)


class Full:
    """One full-size workload resident on the device."""

    def __init__(self, name, tune_fp64):
        pr = make_problem(name, dense=False)
        self.obs, self.sky, self.truth = pr.obs, pr.sky, pr.truth
        obs = self.obs
        self.plan = R.Plan(obs)
        self.dsky = R.DeviceSky.from_host(self.sky)
        shp = (obs.ntime, obs.nbl, obs.nchan, 4)
        say(name, "predict", shp)
        # FP64 model at the evaluation sky (for the chi^2 property) and the data
        self.V64 = self.predict(self.sky, R.FP64)
        g = torch.Generator(device="cuda")
        g.manual_seed(1501)
        truth = self.predict(self.truth, R.FP64)
        nz = torch.randn(shp + (2,), dtype=torch.float64, device="cuda", generator=g) * 0.01
        self.D64 = truth + torch.view_as_complex(nz)
        del truth, nz
        self.W64 = torch.full(shp, 1e4, dtype=torch.float64, device="cuda")
        self.D32, self.W32 = self.D64.to(torch.complex64), self.W64.to(torch.float32)
        for prec in (R.FP64, R.MIXED):
            if prec == R.MIXED or tune_fp64:
                for mode in (R.MODE_CHI2, R.MODE_CHI2_GRAD):
                    D, W = self.data(prec)
                    ws = R.workspace(self.plan, mode, prec, 1, self.sky.nsrc)
                    R.rime_autotune(self.plan, self.dsky, mode, prec, D, W, ws)
                    say(name, "variant", mode, prec,
                        R.rime_variant_info(mode, prec, self.plan.get_variant(mode, prec)))
        torch.cuda.synchronize()

    def data(self, prec):
        return (self.D64, self.W64) if prec == R.FP64 else (self.D32, self.W32)

    def predict(self, sky, prec):
        obs = self.obs
        cdt = torch.complex128 if prec == R.FP64 else torch.complex64
        vis = torch.empty((obs.ntime, obs.nbl, obs.nchan, 4), dtype=cdt, device="cuda")
        ws = R.workspace(self.plan, R.MODE_PREDICT, prec, 1, sky.nsrc)
        R.rime_predict(self.plan, R.DeviceSky.from_host(sky), prec, vis, ws)
        return vis

    def chi2(self, prec, sky=None, grad=False):
        dsky = self.dsky if sky is None else R.DeviceSky.from_host(sky)
        n = self.sky.nsrc if sky is None else sky.nsrc
        D, W = self.data(prec)
        c = torch.empty(1, dtype=torch.float64, device="cuda")
        if grad:
            g = torch.empty((n, 10), dtype=torch.float64, device="cuda")
            ws = R.workspace(self.plan, R.MODE_CHI2_GRAD, prec, 1, n)
            R.rime_chi2_grad(self.plan, dsky, prec, D, W, c, g, ws)
            return c.item(), g.cpu().numpy()
        ws = R.workspace(self.plan, R.MODE_CHI2, prec, 1, n)
        R.rime_chi2(self.plan, dsky, prec, D, W, c, ws)
        return c.item()

    def close(self):
        self.plan.close()


@pytest.fixture(scope="module", params=["c1", "c4"])
def f(request):
    """The workload, built once per module for each name (pytest groups the
    tests by this fixture's parameter)."""
    torch.cuda.empty_cache()
    w = Full(request.param, tune_fp64=(request.param == "c1"))
    w.name = request.param
    yield w
    w.close()
    del w
    torch.cuda.empty_cache()


SAMPLES = {"c1": [(0, 0), (37, 63), (99, 17), (64, 40)],
           "c4": [(0, 255), (11, 0), (19, 131)]}


@pytest.mark.parametrize("prec", [0, 1])
def test_full_predict_sampled(f, prec):
    """Whole (t, channel) slices of the full-size model visibilities against
    the oracle (all baselines, all sources)."""
    name = f.name
    V = f.V64 if prec == R.FP64 else f.predict(f.sky, prec)
    worst = 0.0
    for t, c in SAMPLES[name]:
        o = f.obs.time_slice(t, t + 1).chan_slice(c, c + 1)
        ref = O.model_vis(o, f.sky)[0, :, 0, :]
        got = V[t, :, c, :].cpu().numpy().astype(np.complex128)
        F = O.total_flux(f.sky, o.freq, o.ref_freq)[0]
        err = float(np.abs(got - ref).max() / F)
        worst = max(worst, err)
        say(name, prec, (t, c), f"|dV|/F = {err:.2e}")
    assert worst <= TOL[prec], worst


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_full_chi2_property(f, prec):
    """chi^2 of rime_chi2 and rime_chi2_grad at full size equals
    sum w |V - D|^2 formed from the FP64 model visibilities."""
    name = f.name
    D, W = f.data(prec)
    ref = float((W.double() * (f.V64 - D.to(torch.complex128)).abs() ** 2).sum().item())
    c1 = f.chi2(prec)
    c2, _ = f.chi2(prec, grad=True)
    e1, e2 = abs(c1 - ref) / ref, abs(c2 - ref) / ref
    say(name, prec, f"chi2 {ref:.6e}: chi2-only rel {e1:.2e}, chi2+grad rel {e2:.2e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


def test_full_grad_fp64_directional_fd(f):
    """FP64 gradient at full size against central differences of the FP64
    chi^2 along a random direction per parameter type: direction entries
    +-max(|theta|, 1e-3), steps h and h/2 (h = 1e-7 for l, m, 1e-6 otherwise)
    combined by Richardson extrapolation.  The limit is 1e-6 of sum |g_i d_i|
    plus the rounding noise 64 eps chi^2 / (h/2) and a tenth of the
    difference of the two quotients (the size of the truncation error)."""
    name = f.name
    c0, g = f.chi2(R.FP64, grad=True)
    sky = f.sky
    p0 = sky.params()
    rng = np.random.default_rng(11)
    for k, nm in enumerate(NAMES):
        rows = np.arange(sky.npsrc, sky.nsrc) if k >= 7 else np.arange(sky.nsrc)
        d = np.zeros_like(p0)
        d[rows, k] = np.maximum(np.abs(p0[rows, k]), 1e-3) * rng.choice([-1.0, 1.0], rows.size)
        h = 1e-7 if k < 2 else 1e-6

        def quotient(step):
            v = [f.chi2(R.FP64, sky=Sky.from_params(p0 + sgn * step * d, sky.ngsrc))
                 for sgn in (1, -1)]
            return (v[0] - v[1]) / (2 * step)
        q1, q2 = quotient(h), quotient(h / 2)
        fd = (4 * q2 - q1) / 3
        gd = float(np.sum(g * d))
        scale = float(np.sum(np.abs(g * d)))
        lim = 1e-6 * scale + 64 * 2.2e-16 * c0 / (h / 2) + 0.1 * abs(q1 - q2)
        say(name, nm, f"fd {fd:.6e} g.d {gd:.6e} |diff| {abs(fd - gd):.2e} limit {lim:.2e} "
                      f"(|q1-q2| {abs(q1 - q2):.1e})")
        assert abs(fd - gd) <= lim, (nm, fd, gd, lim)


def test_full_grad_mixed_vs_fp64(f):
    """Mixed-precision gradient at full size against the FP64 gradient, per
    parameter type (2-norm), to the mixed tolerance."""
    name = f.name
    _, g64 = f.chi2(R.FP64, grad=True)
    _, g32 = f.chi2(R.MIXED, grad=True)
    ge = grad_errors(g32, g64, f.sky.npsrc)
    say(name, {k: f"{v:.2e}" for k, v in ge.items()})
    assert max(ge.values()) <= TOL[1], ge
    assert np.all(g32[:f.sky.npsrc, 7:] == 0.0)


def test_full_grad_converged_res64_vs_fp64(f):
    """Converged data at full size (D = the FP64 model at the evaluation sky
    plus noise, rounded to complex64 and given to both precisions): the
    float64-residual mixed gradient against the FP64 gradient, per parameter
    type, to the mixed tolerance.  The float32-mixed gradient's error in this
    regime is printed."""
    name = f.name
    obs = f.obs
    shp = (obs.ntime, obs.nbl, obs.nchan, 4)
    g = torch.Generator(device="cuda")
    g.manual_seed(1502)
    nz = torch.randn(shp + (2,), dtype=torch.float64, device="cuda", generator=g) * 0.01
    Dc32 = (f.V64 + torch.view_as_complex(nz)).to(torch.complex64)
    del nz
    Dc64 = Dc32.to(torch.complex128)
    out = {}
    for prec, (D, W) in ((R.FP64, (Dc64, f.W64)), (R.MIXED_RES64, (Dc32, f.W32)),
                         (R.MIXED, (Dc32, f.W32))):
        c = torch.empty(1, dtype=torch.float64, device="cuda")
        gr = torch.empty((f.sky.nsrc, 10), dtype=torch.float64, device="cuda")
        ws = R.workspace(f.plan, R.MODE_CHI2_GRAD, prec, 1, f.sky.nsrc)
        R.rime_chi2_grad(f.plan, f.dsky, prec, D, W, c, gr, ws)
        out[prec] = (c.item(), gr.cpu().numpy())
        del ws
    del Dc64, Dc32
    c64, g64 = out[R.FP64]
    for prec in (R.MIXED_RES64, R.MIXED):
        cp, gp = out[prec]
        ge = grad_errors(gp, g64, f.sky.npsrc)
        say(name, "converged", prec, f"chi2 rel {abs(cp - c64) / c64:.2e}",
            {k: f"{v:.2e}" for k, v in ge.items()})
        assert abs(cp - c64) <= TOL[1] * c64
        if prec == R.MIXED_RES64:
            assert max(ge.values()) <= TOL[1], ge
