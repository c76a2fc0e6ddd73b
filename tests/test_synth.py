"""The seeded synthetic input generator (the stand-in for the paper's
measurement sets): shapes and sizes of every benchmark configuration,
reproducibility of the seeds, and the moments of the drawn distributions."""
import math

import numpy as np
import pytest

from rime_synth import (ARCSEC, CONFIGS, canonical_baselines, make_batch_problem,
                        make_observation, make_problem, make_sky, rngs)

EXPECTED = {  # name: (na, nbl, ntime, nchan, npsrc, ngsrc, beam, terms per evaluation)
    "c0": (7, 21, 10, 16, 20, 0, False, 6.72e4),
    "c1": (64, 2016, 100, 64, 1000, 500, True, 1.935e10),
    "c2": (64, 2016, 100, 64, 1000, 500, True, 1.935e10),
    "c4": (197, 19306, 20, 256, 1500, 500, True, 1.977e11),
}


@pytest.mark.parametrize("name", sorted(EXPECTED))
def test_config_shapes(name):
    na, nbl, nt, nc, npsrc, ngsrc, beam, terms = EXPECTED[name]
    pr = make_problem(name, dense=False)
    o, s = pr.obs, pr.sky
    assert (o.na, o.nbl, o.ntime, o.nchan) == (na, nbl, nt, nc)
    assert (s.npsrc, s.ngsrc) == (npsrc, ngsrc)
    assert o.beam == beam
    assert o.uvw.shape == (nt, na, 3)
    assert o.freq.shape == (nc,)
    assert abs(nt * nbl * nc * (npsrc + ngsrc) - terms) <= 1e-3 * terms
    if beam:
        assert o.pointing.shape == (nt, na, 2) and o.gains.shape == (na, 2)
    # channels: inclusive linear grid over the configured band
    assert o.freq[0] == CONFIGS[name]["f0"] and o.freq[-1] == CONFIGS[name]["f1"]
    assert np.allclose(np.diff(o.freq), np.diff(o.freq)[0])


def test_dense_arrays():
    pr = make_problem("c0")
    shp = (pr.obs.ntime, pr.obs.nbl, pr.obs.nchan, 4)
    assert pr.noise.shape == shp and pr.noise.dtype == np.complex128
    assert pr.weight.shape == shp and np.all(pr.weight == 1e4)


def test_canonical_baselines():
    p, q = canonical_baselines(5)
    assert list(zip(p, q)) == [(0, 1), (0, 2), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4),
                               (2, 3), (2, 4), (3, 4)]


def test_seeds_reproducible_and_independent():
    a, b = make_problem("c1", ntime=2, nchan=3), make_problem("c1", ntime=2, nchan=3)
    for x, y in ((a.obs.uvw, b.obs.uvw), (a.sky.params(), b.sky.params()),
                 (a.truth.params(), b.truth.params()), (a.noise, b.noise)):
        np.testing.assert_array_equal(x, y)
    c = make_problem("c1", ntime=2, nchan=3, key=99)
    assert not np.array_equal(a.sky.params(), c.sky.params())
    # a time prefix of a configuration is the same track
    long = make_problem("c1", ntime=5, nchan=3)
    np.testing.assert_array_equal(long.obs.uvw[:2], a.obs.uvw)


def test_uvw_rotation():
    pr = make_problem("c1", ntime=50, nchan=1)
    uvw = pr.obs.uvw
    # rotation about w by 0.01 rad per step: |(u, v)| and w are constant in t,
    # the angle advances by 0.01
    r = np.hypot(uvw[..., 0], uvw[..., 1])
    np.testing.assert_allclose(r, r[:1].repeat(50, 0), rtol=1e-12)
    np.testing.assert_array_equal(uvw[..., 2], uvw[:1, :, 2].repeat(50, 0))
    ang = np.unwrap(np.arctan2(uvw[..., 1], uvw[..., 0]), axis=0)
    np.testing.assert_allclose(np.diff(ang, axis=0), 0.01, atol=1e-12)
    assert np.abs(uvw[0, :, :2]).max() <= 1000.0 and np.abs(uvw[0, :, 2]).max() <= 50.0


def test_sky_distributions():
    r = rngs(123)[1]
    s = make_sky(40000, 20000, r)
    n = s.nsrc
    lm = s.lm
    assert np.abs(lm).max() <= 0.02
    assert abs(lm.mean()) < 3e-4 and abs(lm.var() - 0.04 ** 2 / 12) < 2e-6
    lnI = np.log(s.stokes[:, 0])
    assert abs(lnI.mean()) < 0.02 and abs(lnI.std() - 1.0) < 0.02
    frac = s.stokes[:, 1:] / s.stokes[:, :1]
    assert np.abs(frac).max() <= 0.1 and abs(frac.mean()) < 2e-3
    assert abs(s.alpha.mean() + 0.7) < 5e-3 and abs(s.alpha.std() - 0.2) < 5e-3
    el, em, R = s.gshape.T
    tmaj = np.hypot(el, em)
    assert tmaj.min() >= 1.0 * ARCSEC - 1e-18 and tmaj.max() <= 30.0 * ARCSEC + 1e-18
    assert np.all(R <= 1.0) and np.all(R > 1.0 / 30.0 - 1e-12)
    pa = np.arctan2(el, em)  # el = tmaj sin pa, em = tmaj cos pa, pa in [0, pi)
    pa = np.where(pa < 0, pa + math.pi, pa)
    assert abs(pa.mean() - math.pi / 2) < 0.03
    assert n == 60000


def test_instrument_distributions():
    cfg = dict(CONFIGS["c1"], na=2000, ntime=3)
    r = rngs(7)
    o = make_observation(cfg, r[0], r[4])
    assert abs(o.pointing.std() - 1e-4) < 3e-6 and abs(o.pointing.mean()) < 3e-6
    amp, ph = np.abs(o.gains), np.angle(o.gains)
    assert abs(amp.mean() - 1.0) < 3e-3 and abs(amp.std() - 0.05) < 3e-3
    assert abs(ph.mean()) < 6e-3 and abs(ph.std() - 0.1) < 4e-3


def test_perturbation_and_noise():
    pr = make_problem("c1", ntime=20, nchan=8)
    p0, p1 = pr.sky.params(), pr.truth.params()
    ok = p0 != 0  # shape columns of point sources are zero
    rel = p1[ok] / p0[ok] - 1.0
    assert abs(rel.std() - 0.01) < 5e-4 and abs(rel.mean()) < 5e-4
    nz = pr.noise
    assert abs(nz.real.std() - 0.01) < 1e-4 and abs(nz.imag.std() - 0.01) < 1e-4
    assert abs(np.mean(nz.real * nz.imag)) < 1e-6


def test_batch_problem():
    bp = make_batch_problem(nset=64, ntime=2, nchan=2)
    counts = np.array([s.nsrc for s in bp.skies])
    assert counts.min() >= 10 and counts.max() <= 2000 and len(counts) == 64
    for s in bp.skies:
        # each proposal keeps ceil(0.7 n) points and floor(0.3 n) Gaussians of the truth
        n = s.nsrc
        assert s.ngsrc == int(math.floor(0.3 * n))
        rel = s.lm / np.concatenate([bp.truth.lm[:s.npsrc],
                                     bp.truth.lm[bp.truth.npsrc:bp.truth.npsrc + s.ngsrc]]) - 1
        assert np.abs(rel).max() < 0.1
