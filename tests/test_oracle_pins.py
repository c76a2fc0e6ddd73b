"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check is written independently of the oracle's own formulas (numpy
closed forms, brute-force sums, invariants), so that a dropped term, a wrong
sign, a swapped index or a transposed operand in the oracle fails at least one
of them.  ``test_planted_mistakes`` plants such mistakes in the oracle and
confirms that the pins catch each one.
"""
import math

import numpy as np
import pytest

import oracle.rime_oracle as O
from rime_synth import Observation, Sky, canonical_baselines, make_problem

C = 299792458.0


def tiny_obs(na=3, ntime=2, nchan=3, beam=False, gains=False, seed=0, uv=800.0, w=40.0,
             f0=1.3e9, f1=1.5e9):
    rng = np.random.default_rng(seed)
    a1, a2 = canonical_baselines(na)
    uvw = np.empty((ntime, na, 3))
    uvw[..., :2] = rng.uniform(-uv, uv, (ntime, na, 2))
    uvw[..., 2] = rng.uniform(-w, w, (ntime, na))
    obs = Observation(ntime=ntime, na=na, nchan=nchan, ant1=a1, ant2=a2, uvw=uvw,
                      freq=np.linspace(f0, f1, nchan), beam=beam)
    if beam:
        obs.pointing = rng.normal(0, 1e-3, (ntime, na, 2))
    if gains:
        obs.gains = (1 + 0.1 * rng.standard_normal((na, 2))) * np.exp(
            1j * rng.normal(0, 0.3, (na, 2)))
    return obs


def rand_sky(npsrc, ngsrc, seed=1, lm_half=0.02):
    rng = np.random.default_rng(seed)
    n = npsrc + ngsrc
    st = np.empty((n, 4))
    st[:, 0] = rng.uniform(0.5, 3.0, n)
    st[:, 1:] = st[:, :1] * rng.uniform(-0.3, 0.3, (n, 3))
    gs = np.stack([rng.uniform(-1e-4, 1e-4, ngsrc), rng.uniform(-1e-4, 1e-4, ngsrc),
                   rng.uniform(0.2, 1.0, ngsrc)], axis=1) if ngsrc else np.zeros((0, 3))
    return Sky(lm=rng.uniform(-lm_half, lm_half, (n, 2)), stokes=st,
               alpha=rng.normal(-0.7, 0.3, n), gshape=gs)


# --------------------------------------------------------------------------- #
# Individual pins (plain functions so that the planted-mistake test can rerun
# them against a patched oracle)
# --------------------------------------------------------------------------- #

def pin_phase_centre():
    """A source at l = m = 0 with no beam: K = 1 for every antenna, so V = B
    on every baseline (eq. 1 with eq. k_term at n = 1)."""
    obs = tiny_obs(na=4, nchan=5)
    I, Q, U, V, a = 2.0, 0.3, -0.2, 0.1, -0.8
    sky = Sky(lm=np.zeros((1, 2)), stokes=np.array([[I, Q, U, V]]), alpha=np.array([a]))
    vis = O.model_vis(obs, sky)
    f = (obs.freq / obs.ref_freq) ** a
    exp = np.stack([f * (I + Q), f * (U + 1j * V), f * (U - 1j * V), f * (I - Q)], axis=-1)
    np.testing.assert_allclose(vis, np.broadcast_to(exp, vis.shape), rtol=1e-14, atol=1e-14)


def pin_single_point_closed_form():
    """One point source anywhere, no beam: V = B(nu) exp(-2 pi i (du l + dv m
    + dw (n-1)) nu/c) with d = antenna p minus antenna q (eq. k_term)."""
    obs = tiny_obs(na=3, nchan=4, seed=3)
    l, m = 0.013, -0.007
    st = np.array([1.5, 0.2, 0.1, -0.05])
    sky = Sky(lm=np.array([[l, m]]), stokes=st[None], alpha=np.array([0.4]))
    vis = O.model_vis(obs, sky)
    n = math.sqrt(1 - l * l - m * m)
    for t in range(obs.ntime):
        for b, (p, q) in enumerate(zip(obs.ant1, obs.ant2)):
            d = obs.uvw[t, p] - obs.uvw[t, q]
            for c, nu in enumerate(obs.freq):
                ph = np.exp(-2j * np.pi * (d[0] * l + d[1] * m + d[2] * (n - 1)) * nu / C)
                f = (nu / obs.ref_freq) ** 0.4
                B = f * np.array([st[0] + st[1], st[2] + 1j * st[3],
                                  st[2] - 1j * st[3], st[0] - st[1]])
                np.testing.assert_allclose(vis[t, b, c], B * ph, rtol=1e-11, atol=1e-12)


def pin_sign():
    """Sign of the phase: with du > 0, l > 0 small and everything else zero,
    V_xx = I exp(-2 pi i du l nu/c) has a negative imaginary part."""
    uvw = np.zeros((1, 2, 3))
    uvw[0, 0, 0] = 10.0
    obs = Observation(ntime=1, na=2, nchan=1, ant1=np.array([0]), ant2=np.array([1]),
                      uvw=uvw, freq=np.array([1.4e9]))
    sky = Sky(lm=np.array([[1e-3, 0.0]]), stokes=np.array([[1.0, 0, 0, 0]]),
              alpha=np.zeros(1))
    v = O.model_vis(obs, sky)[0, 0, 0, 0]
    n = math.sqrt(1 - 1e-6)
    ang = -2 * math.pi * 10.0 * 1e-3 * 1.4e9 / C
    assert v.imag < 0
    np.testing.assert_allclose(v, complex(math.cos(ang), math.sin(ang)), rtol=1e-13)
    assert abs(n - 1) < 1e-6


def pin_hermitian_swap():
    """Swapping p and q conjugate-transposes every visibility: V_qp = V_pq^H
    (B is Hermitian for real Stokes, eq. brightness_term; the Gaussian shape
    is even in (u, v))."""
    obs = tiny_obs(na=4, nchan=3, beam=True, gains=True, seed=5)
    sky = rand_sky(2, 2, seed=7)
    v = O.model_vis(obs, sky)
    sw = Observation(**{**obs.__dict__, "ant1": obs.ant2.copy(), "ant2": obs.ant1.copy()})
    w = O.model_vis(sw, sky)
    np.testing.assert_allclose(w[..., 0], np.conj(v[..., 0]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(w[..., 1], np.conj(v[..., 2]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(w[..., 2], np.conj(v[..., 1]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(w[..., 3], np.conj(v[..., 3]), rtol=1e-12, atol=1e-13)


def pin_zero_width_gaussian():
    """A Gaussian of zero width (el = em = 0, any R) is a point source."""
    obs = tiny_obs(na=4, nchan=3, beam=True, gains=True, seed=6)
    sk = rand_sky(0, 2, seed=8)
    sk.gshape[:, 0:2] = 0.0
    pt = Sky(lm=sk.lm, stokes=sk.stokes, alpha=sk.alpha)
    np.testing.assert_allclose(O.model_vis(obs, sk), O.model_vis(obs, pt), rtol=1e-14,
                               atol=1e-14)


def pin_gaussian_dft():
    """The shape factor equals a brute-force 2-D Fourier sum of the sky-plane
    elliptical Gaussian (FWHM axes, position angle from +m towards +l),
    normalised to unit integrated flux."""
    tmaj, tmin, pa = 2.0e-4, 0.9e-4, 0.6
    el, em, R = tmaj * math.sin(pa), tmaj * math.cos(pa), tmin / tmaj
    h = 8 * tmaj
    x = np.linspace(-h, h, 801)
    L, M = np.meshgrid(x, x, indexing="ij")
    xmaj = L * math.sin(pa) + M * math.cos(pa)
    xmin = L * math.cos(pa) - M * math.sin(pa)
    img = np.exp(-4 * math.log(2) * ((xmaj / tmaj) ** 2 + (xmin / tmin) ** 2))
    freq = np.array([1.4e9])
    import torch
    for (u, v) in [(1500.0, 0.0), (-700.0, 2100.0), (300.0, -900.0), (2500., 2500.)]:
        uw, vw = u * 1.4e9 / C, v * 1.4e9 / C
        ft = np.sum(img * np.exp(-2j * np.pi * (uw * L + vw * M))) / np.sum(img)
        duvw = torch.tensor([[[u, v, 0.0]]], dtype=torch.float64)
        gs = torch.tensor([[el, em, R]], dtype=torch.float64)
        S = O.gauss_shape(duvw, gs, torch.tensor(freq))[0, 0, 0, 0].item()
        assert abs(ft.imag) < 1e-12
        np.testing.assert_allclose(S, ft.real, rtol=1e-9, atol=1e-12)


def pin_gaussian_half_power():
    """Along the major axis, u' theta_maj = 2 ln 2 / pi gives S = 1/2, and
    u' theta_maj = 1 gives exp(-pi^2 / (4 ln 2)); along the minor axis the
    same holds with theta_min."""
    import torch
    tmaj, tmin, pa = 3e-5, 1e-5, 1.1
    gs = torch.tensor([[tmaj * math.sin(pa), tmaj * math.cos(pa), tmin / tmaj]],
                      dtype=torch.float64)
    nu = 1.4e9
    for rho, theta, dirv, expect in [
        (2 * math.log(2) / math.pi / tmaj, tmaj, (math.sin(pa), math.cos(pa)), 0.5),
        (1.0 / tmaj, tmaj, (math.sin(pa), math.cos(pa)), math.exp(-math.pi ** 2 / (4 * math.log(2)))),
        (2 * math.log(2) / math.pi / tmin, tmin, (math.cos(pa), -math.sin(pa)), 0.5),
    ]:
        u, v = rho * dirv[0] * C / nu, rho * dirv[1] * C / nu
        S = O.gauss_shape(torch.tensor([[[u, v, 0.0]]], dtype=torch.float64), gs,
                          torch.tensor([nu], dtype=torch.float64))[0, 0, 0, 0].item()
        np.testing.assert_allclose(S, expect, rtol=1e-12)


def pin_beam_values():
    """Beam factor: e = 1 at the pointing centre; beyond the clip radius the
    factor is the floor cos^3(1.0881) = 0.1000066 (to 7 digits); in between
    e = cos^3(65 r nu / 1.4 GHz)."""
    import torch
    lm = torch.tensor([[0.0, 0.0], [0.03, 0.0], [0.003, 0.004]], dtype=torch.float64)
    pnt = torch.zeros((1, 1, 2), dtype=torch.float64)
    freq = torch.tensor([1.4e9, 1.0e9], dtype=torch.float64)
    e = O.beam_e(lm, pnt, freq, 65.0, 1.4e9, 1.0881)[0, 0].numpy()
    np.testing.assert_allclose(e[0], [1.0, 1.0], rtol=0, atol=0)
    assert abs(e[1, 0] - 0.1000066) < 5e-8 and abs(e[1, 1] - 0.1000066) < 5e-8
    r = 0.005
    np.testing.assert_allclose(e[2], [math.cos(65 * r) ** 3, math.cos(65 * r / 1.4) ** 3],
                               rtol=1e-14)


def pin_spectral():
    """alpha = 0 gives a flat spectrum; nu = nu_ref gives factor 1 for any alpha."""
    import torch
    f = O.spectral(torch.tensor([0.0, -0.7, 2.0], dtype=torch.float64),
                   torch.tensor([0.9e9, 1.4e9, 1.7e9], dtype=torch.float64), 1.4e9).numpy()
    np.testing.assert_allclose(f[0], 1.0, rtol=0)
    np.testing.assert_allclose(f[:, 1], 1.0, rtol=0)
    np.testing.assert_allclose(f[2, 2], (1.7 / 1.4) ** 2, rtol=1e-15)


def pin_gain_placement():
    """Gains sit in E: a phase-centre source gives V_ij = g_pi conj(g_qj) B_ij."""
    obs = tiny_obs(na=3, nchan=2, gains=True, seed=9)
    st = np.array([1.0, 0.25, -0.5, 0.75])
    sky = Sky(lm=np.zeros((1, 2)), stokes=st[None], alpha=np.zeros(1))
    v = O.model_vis(obs, sky)
    B = np.array([[st[0] + st[1], st[2] + 1j * st[3]], [st[2] - 1j * st[3], st[0] - st[1]]])
    for b, (p, q) in enumerate(zip(obs.ant1, obs.ant2)):
        gp, gq = obs.gains[p], obs.gains[q]
        exp = np.array([[gp[i] * np.conj(gq[j]) * B[i, j] for j in range(2)] for i in range(2)])
        np.testing.assert_allclose(v[0, b, 0], exp.reshape(4), rtol=1e-13)


def pin_brute_force():
    """The vectorised oracle equals eq. 1 with scalar loops on a 3-antenna
    problem with beam, gains, one point and one Gaussian source."""
    obs = tiny_obs(na=3, ntime=2, nchan=3, beam=True, gains=True, seed=11)
    sky = rand_sky(1, 1, seed=12)
    np.testing.assert_allclose(O.model_vis(obs, sky), O.brute_force_vis(obs, sky),
                               rtol=1e-11, atol=1e-12)


def pin_phase_exact_fraction():
    """The phase fraction of eq. k_term equals the exact fraction of
    (u l + v m + w (n - 1)) nu / c over the float64 inputs, evaluated in
    rational arithmetic, to 1e-15 turns at phases of about a thousand turns
    (u, v up to 8 km as on the large array, 1.76 GHz)."""
    import torch
    from fractions import Fraction as Fr
    rng = np.random.default_rng(9)
    uvw = rng.uniform(-8000.0, 8000.0, (2, 4, 3))
    uvw[..., 2] /= 40.0
    lm = rng.uniform(-0.03, 0.03, (5, 2))
    freq = np.linspace(0.95e9, 1.76e9, 3)
    r = O.phase_turns(torch.tensor(uvw), torch.tensor(lm), torch.tensor(freq)).numpy()
    nm1 = O.n_minus_one(torch.tensor(lm[:, 0]), torch.tensor(lm[:, 1])).numpy()
    big = 0.0
    for t in range(2):
        for a in range(4):
            for s in range(5):
                tau = (Fr(uvw[t, a, 0]) * Fr(lm[s, 0]) + Fr(uvw[t, a, 1]) * Fr(lm[s, 1])
                       + Fr(uvw[t, a, 2]) * Fr(float(nm1[s])))
                for f in range(3):
                    x = tau * Fr(float(freq[f] / C))
                    frac = x - round(x)
                    big = max(big, abs(float(x)))
                    assert abs(r[t, a, s, f] - float(frac)) <= 1e-15, (t, a, s, f)
    assert big > 300.0


PINS = [pin_phase_centre, pin_single_point_closed_form, pin_sign, pin_hermitian_swap,
        pin_zero_width_gaussian, pin_gaussian_dft, pin_gaussian_half_power,
        pin_beam_values, pin_spectral, pin_gain_placement, pin_brute_force,
        pin_phase_exact_fraction]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


# --------------------------------------------------------------------------- #
# Invariants of the sum and of chi-squared
# --------------------------------------------------------------------------- #

def test_linear_in_stokes_and_additive_over_sources():
    """V is linear in each source's (I, Q, U, V) and additive over sources
    (the source sum of Section 2.1)."""
    obs = tiny_obs(na=4, nchan=3, beam=True, gains=True, seed=13)
    sky = rand_sky(2, 2, seed=14)
    v = O.model_vis(obs, sky)
    s2 = Sky(lm=sky.lm, stokes=2.5 * sky.stokes, alpha=sky.alpha, gshape=sky.gshape)
    np.testing.assert_allclose(O.model_vis(obs, s2), 2.5 * v, rtol=1e-13, atol=1e-13)
    parts = [sky.subset(2, 0), Sky(lm=sky.lm[2:], stokes=sky.stokes[2:], alpha=sky.alpha[2:],
                                   gshape=sky.gshape)]
    np.testing.assert_allclose(O.model_vis(obs, parts[0]) + O.model_vis(obs, parts[1]), v,
                               rtol=1e-12, atol=1e-13)


def test_chi2_invariants():
    """chi^2 = 0 when D = V; linear in w; additive over time chunks (the
    paper's subdivision along time)."""
    obs = tiny_obs(na=4, ntime=3, nchan=3, beam=True, gains=True, seed=15)
    sky = rand_sky(2, 1, seed=16)
    v = O.model_vis(obs, sky)
    w = np.random.default_rng(0).uniform(0.5, 2.0, v.shape)
    assert O.chi2(obs, sky, v, w) == 0.0
    D = v + 0.1 * (np.random.default_rng(1).standard_normal(v.shape) + 1j)
    c = O.chi2(obs, sky, D, w)
    np.testing.assert_allclose(O.chi2(obs, sky, D, 3.0 * w), 3.0 * c, rtol=1e-14)
    parts = sum(O.chi2(obs.time_slice(t, t + 1), sky, D[t:t + 1], w[t:t + 1])
                for t in range(obs.ntime))
    np.testing.assert_allclose(parts, c, rtol=1e-13)
    # direct definition, one term at a time
    ref = sum(w.flat[i] * abs(v.flat[i] - D.flat[i]) ** 2 for i in range(v.size))
    np.testing.assert_allclose(c, ref, rtol=1e-13)


def test_loglike_const():
    w = np.array([1.0, 2.0, 4.0])
    np.testing.assert_allclose(O.loglike_const(w), sum(math.log(2 * math.pi / x) for x in w))


def test_total_flux():
    sky = rand_sky(3, 0, seed=2)
    f = O.total_flux(sky, np.array([1.4e9, 0.7e9]), 1.4e9)
    np.testing.assert_allclose(f[0], sky.stokes[:, 0].sum())
    np.testing.assert_allclose(f[1], (sky.stokes[:, 0] * 0.5 ** sky.alpha).sum())


# --------------------------------------------------------------------------- #
# Gradient: autograd of the oracle against central finite differences
# --------------------------------------------------------------------------- #

def _fd_problem(seed=21):
    obs = tiny_obs(na=4, ntime=2, nchan=3, beam=True, gains=True, seed=seed)
    sky = rand_sky(2, 2, seed=seed + 1)
    truth = Sky.from_params(sky.params() * (1 + 0.02 * np.random.default_rng(seed).standard_normal(
        (sky.nsrc, 10))), sky.ngsrc)
    D = O.model_vis(obs, truth) + 0.01 * (1 + 1j)
    W = np.full(D.shape, 1e4)
    return obs, sky, D, W


def test_grad_matches_central_fd():
    obs, sky, D, W = _fd_problem()
    c, g = O.chi2_and_grad(obs, sky, D, W)
    np.testing.assert_allclose(c, O.chi2(obs, sky, D, W), rtol=1e-13)
    p0 = sky.params()
    for s in range(sky.nsrc):
        for k in range(10):
            if k >= 7 and s < sky.npsrc:
                assert g[s, k] == 0.0
                continue
            h = 1e-6 * max(abs(p0[s, k]), 1e-3)
            pp, pm = p0.copy(), p0.copy()
            pp[s, k] += h
            pm[s, k] -= h
            fd = (O.chi2(obs, Sky.from_params(pp, sky.ngsrc), D, W)
                  - O.chi2(obs, Sky.from_params(pm, sky.ngsrc), D, W)) / (2 * h)
            assert abs(fd - g[s, k]) <= 1e-6 * max(abs(g[s, k]), 1e-3 * np.abs(g).max()), \
                (s, k, fd, g[s, k])


# --------------------------------------------------------------------------- #
# Planted mistakes: each one must make at least one pin fail
# --------------------------------------------------------------------------- #

def _mut_sign(monkeypatch):
    orig = O.phase_turns
    monkeypatch.setattr(O, "phase_turns", lambda *a: -orig(*a))


def _mut_plain_phase(monkeypatch):
    # the phase as plain float64 products and sums (rounded), not error-free
    def pt(uvw, lm, freq):
        nm1 = O.n_minus_one(lm[:, 0], lm[:, 1])
        tau = (uvw[..., 0][..., None] * lm[:, 0] + uvw[..., 1][..., None] * lm[:, 1]
               + uvw[..., 2][..., None] * nm1)
        x = tau[..., None] * (freq / O.C_LIGHT)
        return x - torch.round(x)
    import torch
    monkeypatch.setattr(O, "phase_turns", pt)


def _mut_drop_w(monkeypatch):
    def pt(uvw, lm, freq):
        u2 = uvw.clone()
        u2[..., 2] = 0.0
        return O_phase_turns(u2, lm, freq)
    O_phase_turns = O.phase_turns
    monkeypatch.setattr(O, "phase_turns", pt)


def _mut_transpose_B(monkeypatch):
    orig = O.brightness
    monkeypatch.setattr(O, "brightness", lambda *a: orig(*a).transpose(-1, -2))


def _mut_half_B(monkeypatch):
    orig = O.brightness
    monkeypatch.setattr(O, "brightness", lambda *a: 0.5 * orig(*a))


def _mut_alpha_sign(monkeypatch):
    orig = O.spectral
    monkeypatch.setattr(O, "spectral", lambda a, f, r: orig(-a, f, r))


def _mut_gauss_swap(monkeypatch):
    orig = O.gauss_shape

    def gs(duvw, g, freq):
        g2 = g[:, [1, 0, 2]]
        return orig(duvw, g2, freq)
    monkeypatch.setattr(O, "gauss_shape", gs)


def _mut_gauss_R(monkeypatch):
    orig = O.gauss_shape

    def gs(duvw, g, freq):
        g2 = g.clone()
        g2[:, 2] = 1.0
        return orig(duvw, g2, freq)
    monkeypatch.setattr(O, "gauss_shape", gs)


def _mut_beam_square(monkeypatch):
    orig = O.beam_e
    monkeypatch.setattr(O, "beam_e", lambda *a: orig(*a) ** (2.0 / 3.0))


def _mut_beam_noclip(monkeypatch):
    orig = O.beam_e
    monkeypatch.setattr(O, "beam_e", lambda lm, p, f, k, r, clip: orig(lm, p, f, k, r, 10.0))


def _mut_gain_conj(monkeypatch):
    orig = O.jones_A

    def ja(ot, lm, freq):
        ot = dict(ot)
        if ot["gains"] is not None:
            ot["gains"] = ot["gains"].conj()
        return orig(ot, lm, freq)
    monkeypatch.setattr(O, "jones_A", ja)


MUTATIONS = [_mut_sign, _mut_plain_phase, _mut_drop_w, _mut_transpose_B, _mut_half_B, _mut_alpha_sign,
             _mut_gauss_swap, _mut_gauss_R, _mut_beam_square, _mut_beam_noclip,
             _mut_gain_conj]


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m.__name__ for m in MUTATIONS])
def test_planted_mistakes(mut, monkeypatch):
    mut(monkeypatch)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutation {mut.__name__}"


def test_synth_config_c0_shapes():
    pr = make_problem("c0")
    assert pr.obs.nbl == 21 and pr.obs.uvw.shape == (10, 7, 3)
    assert pr.sky.nsrc == 20 and pr.sky.ngsrc == 0
    assert pr.noise.shape == (10, 21, 16, 4)
    np.testing.assert_allclose(pr.obs.freq[[0, -1]], [1.36e9, 1.44e9])


def test_domain_error():
    """Directions with l^2 + m^2 >= 1 are outside the domain of
    n = sqrt(1 - l^2 - m^2) (Section 2.1): the oracle refuses them."""
    obs = tiny_obs()
    sky = Sky(lm=np.array([[0.8, 0.6]]), stokes=np.array([[1.0, 0, 0, 0]]), alpha=np.zeros(1))
    with pytest.raises(ValueError):
        O.model_vis(obs, sky)


# --------------------------------------------------------------------------- #
# The pointing centre, the direction-independent term G, exponential disks and
# brightness per timestep
# --------------------------------------------------------------------------- #

def _fd(f, x0, h):
    return (f(x0 + h) - f(x0 - h)) / (2 * h)


def test_beam_gradient_at_pointing_centre():
    """A source exactly on the pointing centres (r = 0): e = cos^3(k r nu/nu_b)
    is smooth there, so the gradient with respect to l and m is finite and
    equals central differences (the beam part of it is 0)."""
    obs = tiny_obs(na=4, nchan=3, beam=True, seed=5)
    obs.pointing = np.zeros_like(obs.pointing)
    sky = Sky(lm=np.zeros((1, 2)), stokes=np.array([[2.0, 0.3, -0.2, 0.1]]),
              alpha=np.array([-0.5]))
    rng = np.random.default_rng(6)
    D = O.model_vis(obs, sky) + 0.05 * (rng.standard_normal((2, 6, 3, 4))
                                        + 1j * rng.standard_normal((2, 6, 3, 4)))
    W = np.full(D.shape, 1e2)
    c, g = O.chi2_and_grad(obs, sky, D, W)
    assert np.all(np.isfinite(g))
    for k in (0, 1):
        def f(x):
            p = sky.params()
            p[0, k] = x
            return O.chi2(obs, Sky.from_params(p, 0), D, W)
        fd = _fd(f, 0.0, 1e-8)
        assert abs(fd - g[0, k]) <= 1e-6 * max(abs(g[0, k]), 1.0), (k, fd, g[0, k])


def _rand_die(rng, T, A, F):
    g = (1 + 0.1 * rng.standard_normal((T, A, F, 2, 2))) * np.exp(
        1j * rng.normal(0, 0.3, (T, A, F, 2, 2)))
    g[..., 0, 1] *= 0.1
    g[..., 1, 0] *= 0.1
    return g


def test_die_identity_and_closed_form():
    """G = 1 reproduces the model; for one source at the phase centre with no
    beam and unit gains the coherency is B, so V_pq = G_p B G_q^H (eq. 1),
    written out with numpy; the p <-> q swap gives the Hermitian transpose."""
    obs = tiny_obs(na=4, nchan=3, seed=7)
    sky = rand_sky(3, 1, seed=8)
    eye = np.broadcast_to(np.eye(2, dtype=complex), (2, 4, 3, 2, 2)).copy()
    np.testing.assert_array_equal(O.model_vis(obs, sky, die=eye), O.model_vis(obs, sky))
    rng = np.random.default_rng(9)
    G = _rand_die(rng, 2, 4, 3)
    I, Q, U, V, a = 1.7, 0.2, -0.3, 0.05, -0.6
    one = Sky(lm=np.zeros((1, 2)), stokes=np.array([[I, Q, U, V]]), alpha=np.array([a]))
    vis = O.model_vis(obs, one, die=G)
    f = (obs.freq / obs.ref_freq) ** a
    B = np.zeros((3, 2, 2), dtype=complex)
    B[:, 0, 0], B[:, 0, 1], B[:, 1, 0], B[:, 1, 1] = f * (I + Q), f * (U + 1j * V), \
        f * (U - 1j * V), f * (I - Q)
    for t in range(2):
        for b, (p, q) in enumerate(zip(obs.ant1, obs.ant2)):
            for c in range(3):
                exp = G[t, p, c] @ B[c] @ G[t, q, c].conj().T
                np.testing.assert_allclose(vis[t, b, c], exp.reshape(4), rtol=1e-13, atol=1e-13)
    sw = Observation(**{**obs.__dict__, "ant1": obs.ant2, "ant2": obs.ant1})
    vs = O.model_vis(sw, sky, die=G).reshape(2, 6, 3, 2, 2)
    vv = O.model_vis(obs, sky, die=G).reshape(2, 6, 3, 2, 2)
    np.testing.assert_allclose(vs, vv.conj().swapaxes(-1, -2), rtol=1e-13, atol=1e-13)


def test_die_gradient_matches_central_fd():
    """d chi^2 / d Re G + i d chi^2 / d Im G from autograd against central
    differences of chi^2 in the real and imaginary part of single entries."""
    obs = tiny_obs(na=3, nchan=2, beam=True, gains=True, seed=10)
    obs.pointing = np.random.default_rng(1).normal(0, 1e-3, (2, 3, 2))
    sky = rand_sky(2, 1, seed=11)
    rng = np.random.default_rng(12)
    G = _rand_die(rng, 2, 3, 2)
    D = O.model_vis(obs, sky, die=_rand_die(rng, 2, 3, 2))
    W = np.full(D.shape, 3.0)
    r = O.chi2_and_grad_ext(obs, sky, D, W, die=G)
    gd = r["grad_die"]
    assert abs(r["chi2"] - O.chi2_from_vis(O.model_vis(obs, sky, die=G), D, W)) <= 1e-12 * r["chi2"]
    for idx in [(0, 0, 0, 0, 0), (1, 2, 1, 0, 1), (0, 1, 1, 1, 0), (1, 0, 0, 1, 1)]:
        for part, unit in ((np.real, 1.0), (np.imag, 1j)):
            def f(x):
                G2 = G.copy()
                G2[idx] += unit * x
                return O.chi2_from_vis(O.model_vis(obs, sky, die=G2), D, W)
            fd = _fd(f, 0.0, 1e-6)
            assert abs(fd - part(gd[idx])) <= 1e-6 * max(abs(gd[idx]), 1.0), (idx, fd, gd[idx])


def _disk_dft(u, v, h, R, pa, n=3200, extent=40.0):
    """Normalised 2-D transform of exp(-sqrt((x/h)^2 + (y/(R h))^2)) with x the
    major axis at position angle pa (from +m towards +l), by a direct sum on a
    grid of the principal axes (spacing h extent 2 / n and R times that)."""
    x = (np.arange(n) - (n - 1) / 2) * (2 * extent * h / n)
    y = x * R
    prof = np.exp(-np.sqrt((x[:, None] / h) ** 2 + (y[None, :] / (R * h)) ** 2))
    kx = u * math.sin(pa) + v * math.cos(pa)       # along the major axis
    ky = u * math.cos(pa) - v * math.sin(pa)       # along the minor axis
    ex = np.exp(-2j * math.pi * kx * x)
    ey = np.exp(-2j * math.pi * ky * y)
    return (ex @ prof @ ey) / prof.sum()


def test_disk_shape_is_the_profile_transform():
    """The exponential-disk shape factor equals a direct 2-D transform of the
    sky-plane profile (reading of the Sersic index-1 morphology)."""
    import torch
    h, R, pa = 1.0, 0.55, 0.7
    for (u, v) in [(0.0, 0.0), (0.05, 0.02), (0.1, -0.2), (-0.25, 0.15), (0.4, 0.3)]:
        ref = _disk_dft(u, v, h, R, pa)
        xs = torch.tensor([[h * math.sin(pa), h * math.cos(pa), R]], dtype=torch.float64)
        # duvw in metres with nu / c = 1
        duvw = torch.tensor([[[u, v, 0.0]]], dtype=torch.float64)
        got = O.disk_shape(duvw, xs, torch.tensor([O.C_LIGHT], dtype=torch.float64))
        assert abs(float(got.reshape(-1)[0]) - ref.real) <= 2e-6, (u, v, float(got), ref)
        assert abs(ref.imag) <= 1e-9


def test_disk_limits_and_gradient():
    """A zero-size disk is a point source; the shape gradient matches central
    differences."""
    obs = tiny_obs(na=4, nchan=3, beam=True, gains=True, seed=13)
    obs.pointing = np.random.default_rng(2).normal(0, 1e-3, (2, 4, 2))
    base = rand_sky(3, 0, seed=14)
    xs = np.array([[2e-5, -1e-5, 0.6]])
    disk = Sky(lm=base.lm, stokes=base.stokes, alpha=base.alpha, xshape=np.zeros((1, 3)))
    np.testing.assert_allclose(O.model_vis(obs, disk), O.model_vis(obs, base), rtol=0, atol=1e-14)
    disk = Sky(lm=base.lm, stokes=base.stokes, alpha=base.alpha, xshape=xs)
    assert disk.nxsrc == 1 and disk.npsrc == 2
    D = O.model_vis(obs, Sky.from_params(disk.params() * 1.01, 0, 1))
    W = np.full(D.shape, 5.0)
    c, g = O.chi2_and_grad(obs, disk, D, W)
    for k in (7, 8, 9):
        def f(x):
            p = disk.params()
            p[2, k] = x
            return O.chi2(obs, Sky.from_params(p, 0, 1), D, W)
        x0 = disk.params()[2, k]
        fd = _fd(f, x0, 1e-6 * abs(x0))
        assert abs(fd - g[2, k]) <= 1e-6 * max(abs(g[2, k]), 1e-3 * np.abs(g).max()), (k, fd, g[2, k])


def test_brightness_per_timestep():
    """Brightness per timestep (Table rime_input's ntime x nsrc array): a
    constant one reproduces the static model and gradient; timestep t depends
    only on stokes_t[t]; its gradient matches central differences."""
    obs = tiny_obs(na=4, nchan=3, beam=True, gains=True, seed=15)
    obs.pointing = np.random.default_rng(3).normal(0, 1e-3, (2, 4, 2))
    sky = rand_sky(2, 1, seed=16)
    st_c = np.broadcast_to(sky.stokes, (2,) + sky.stokes.shape).copy()
    np.testing.assert_array_equal(O.model_vis(obs, sky, stokes_t=st_c), O.model_vis(obs, sky))
    rng = np.random.default_rng(17)
    st = sky.stokes[None] * (1 + 0.1 * rng.standard_normal((2, 3, 4)))
    vis = O.model_vis(obs, sky, stokes_t=st)
    for t in range(2):
        s_t = Sky(lm=sky.lm, stokes=st[t], alpha=sky.alpha, gshape=sky.gshape)
        np.testing.assert_array_equal(vis[t], O.model_vis(obs.time_slice(t, t + 1), s_t)[0])
    D = O.model_vis(obs, sky) + 0.01 * rng.standard_normal(vis.shape)
    W = np.full(D.shape, 1e2)
    r = O.chi2_and_grad_ext(obs, sky, D, W, stokes_t=st)
    c0, g0 = O.chi2_and_grad(obs, sky, D, W)
    r0 = O.chi2_and_grad_ext(obs, sky, D, W, stokes_t=st_c)
    np.testing.assert_allclose(r0["grad"], g0, rtol=1e-12, atol=1e-12 * np.abs(g0).max())
    gs = r["grad_stokes_t"]
    for idx in [(0, 0, 0), (1, 2, 1), (0, 1, 3), (1, 0, 2)]:
        def f(x):
            s2 = st.copy()
            s2[idx] = x
            return O.chi2_from_vis(O.model_vis(obs, sky, stokes_t=s2), D, W)
        fd = _fd(f, st[idx], 1e-6 * abs(st[idx]))
        assert abs(fd - gs[idx]) <= 1e-6 * max(abs(gs[idx]), 1e-3 * np.abs(gs).max()), (idx, fd)


# planted mistakes in the extensions: each must fail one of their pins
EXT_PINS = [test_beam_gradient_at_pointing_centre, test_die_identity_and_closed_form,
            test_die_gradient_matches_central_fd, test_disk_shape_is_the_profile_transform,
            test_disk_limits_and_gradient, test_brightness_per_timestep]


def _mut_die_no_conj(monkeypatch):
    def ad(vis, G, ant1, ant2):
        a1 = np.asarray(ant1, dtype=np.int64)
        a2 = np.asarray(ant2, dtype=np.int64)
        return G[:, a1] @ vis @ G[:, a2].transpose(-1, -2)
    monkeypatch.setattr(O, "apply_die", ad)


def _mut_die_order(monkeypatch):
    def ad(vis, G, ant1, ant2):
        a1 = np.asarray(ant1, dtype=np.int64)
        a2 = np.asarray(ant2, dtype=np.int64)
        return G[:, a2] @ vis @ G[:, a1].conj().transpose(-1, -2)
    monkeypatch.setattr(O, "apply_die", ad)


def _mut_disk_exponent(monkeypatch):
    orig = O.disk_shape
    monkeypatch.setattr(O, "disk_shape", lambda *a: orig(*a) ** (2.0 / 3.0))


def _mut_disk_axes(monkeypatch):
    orig = O.disk_shape

    def ds(duvw, xs, freq):
        x2 = xs.clone()
        x2[:, 2] = 1.0
        return orig(duvw, x2, freq)
    monkeypatch.setattr(O, "disk_shape", ds)


def _mut_beam_nan_centre(monkeypatch):
    def be(lm, pointing, freq, k, ref, clip):
        import torch
        dl = lm[None, None, :, 0] - pointing[..., 0][..., None]
        dm = lm[None, None, :, 1] - pointing[..., 1][..., None]
        r = torch.sqrt(dl * dl + dm * dm)
        return torch.cos(torch.clamp(k * r[..., None] * (freq / ref), max=clip)) ** 3
    monkeypatch.setattr(O, "beam_e", be)


EXT_MUTATIONS = [_mut_die_no_conj, _mut_die_order, _mut_disk_exponent, _mut_disk_axes,
                 _mut_beam_nan_centre]


@pytest.mark.parametrize("mut", EXT_MUTATIONS, ids=[m.__name__ for m in EXT_MUTATIONS])
def test_planted_mistakes_extensions(mut, monkeypatch):
    mut(monkeypatch)
    failed = []
    for pin in EXT_PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutation {mut.__name__}"
