"""Seeded synthetic observations and sky models for the RIME chi-squared engine.

This module only draws random numbers and arranges them into arrays; it holds
none of the measurement-equation arithmetic.  Both the HIP library (through its
Python binding) and the CPU oracle consume what it produces.  Model
visibilities for the "observed" data are composed by the caller (the oracle in
tests, the GPU in benchmarks) from ``truth`` parameters plus :func:`noise`.

Array conventions (all float64 / complex128 numpy arrays):

* ``uvw``      [ntime][na][3]   per-antenna u, v, w in metres
* ``freq``     [nchan]          channel frequencies in Hz
* ``ant1/ant2``[nbl]            baseline antenna indices, p < q, row-major
* ``pointing`` [ntime][na][2]   per-antenna pointing error (dl, dm) in rad
* ``gains``    [na][2]          diagonal complex gain per antenna and feed
* ``lm``       [nsrc][2]        direction cosines; point sources first
* ``stokes``   [nsrc][4]        I, Q, U, V in Jy at the reference frequency
* ``alpha``    [nsrc]           spectral index
* ``gshape``   [ngsrc][3]       Gaussian (el, em, R) for the ngsrc sources after
                                the points: el = theta_maj sin(pa),
                                em = theta_maj cos(pa), R = theta_min/theta_maj
* ``xshape``   [nxsrc][3]       exponential-disk (el, em, R) for the trailing
                                nxsrc sources: el = h sin(pa), em = h cos(pa),
                                h the major-axis scale length, R the axis ratio
* data / weight [ntime][nbl][nchan][4] with correlations (xx, xy, yx, yy)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ARCSEC = math.pi / (180.0 * 3600.0)
BASE_SEED = 150107719

# Workload recipes: the five configurations of the benchmark plan.
CONFIGS = {
    # plain FP64, point sources only, no beam
    "c0": dict(na=7, ntime=10, nchan=16, f0=1.36e9, f1=1.44e9, npsrc=20, ngsrc=0,
               beam=False, uv_half=1000.0, w_half=50.0),
    # full RIME: point + Gaussian sources, cos^3 beam with pointing and gains
    "c1": dict(na=64, ntime=100, nchan=64, f0=0.9e9, f1=1.7e9, npsrc=1000, ngsrc=500,
               beam=True, uv_half=1000.0, w_half=50.0),
    # same observation as c1, evaluated with the adjoint
    "c2": dict(na=64, ntime=100, nchan=64, f0=0.9e9, f1=1.7e9, npsrc=1000, ngsrc=500,
               beam=True, uv_half=1000.0, w_half=50.0),
    # batched proposals over one shared observation
    "c3": dict(na=64, ntime=50, nchan=32, f0=0.9e9, f1=1.7e9, npsrc=1400, ngsrc=600,
               beam=True, uv_half=1000.0, w_half=50.0, nset=256, nmin=10, nmax=2000,
               gfrac=0.3),
    # large array
    "c4": dict(na=197, ntime=20, nchan=256, f0=0.95e9, f1=1.76e9, npsrc=1500, ngsrc=500,
               beam=True, uv_half=8000.0, w_half=200.0),
}

REF_FREQ = 1.4e9
BEAM_K = 65.0
BEAM_REF_FREQ = 1.4e9
BEAM_CLIP = 1.0881
NOISE_SIGMA = 0.01
PERTURB_FRAC = 0.01
ROT_PER_STEP = 0.01


@dataclass
class Observation:
    ntime: int
    na: int
    nchan: int
    ant1: np.ndarray
    ant2: np.ndarray
    uvw: np.ndarray
    freq: np.ndarray
    ref_freq: float = REF_FREQ
    beam: bool = False
    pointing: np.ndarray | None = None
    gains: np.ndarray | None = None
    beam_k: float = BEAM_K
    beam_ref_freq: float = BEAM_REF_FREQ
    beam_clip: float = BEAM_CLIP

    @property
    def nbl(self) -> int:
        return int(self.ant1.shape[0])

    def time_slice(self, t0: int, t1: int) -> "Observation":
        """The same observation restricted to timesteps [t0, t1)."""
        return Observation(
            ntime=t1 - t0, na=self.na, nchan=self.nchan, ant1=self.ant1, ant2=self.ant2,
            uvw=self.uvw[t0:t1].copy(), freq=self.freq, ref_freq=self.ref_freq,
            beam=self.beam,
            pointing=None if self.pointing is None else self.pointing[t0:t1].copy(),
            gains=self.gains, beam_k=self.beam_k, beam_ref_freq=self.beam_ref_freq,
            beam_clip=self.beam_clip)

    def chan_slice(self, c0: int, c1: int) -> "Observation":
        """The same observation restricted to channels [c0, c1)."""
        return Observation(
            ntime=self.ntime, na=self.na, nchan=c1 - c0, ant1=self.ant1, ant2=self.ant2,
            uvw=self.uvw, freq=self.freq[c0:c1].copy(), ref_freq=self.ref_freq,
            beam=self.beam, pointing=self.pointing, gains=self.gains,
            beam_k=self.beam_k, beam_ref_freq=self.beam_ref_freq,
            beam_clip=self.beam_clip)


@dataclass
class Sky:
    lm: np.ndarray
    stokes: np.ndarray
    alpha: np.ndarray
    gshape: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    xshape: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))

    @property
    def nsrc(self) -> int:
        return int(self.lm.shape[0])

    @property
    def ngsrc(self) -> int:
        return int(self.gshape.shape[0])

    @property
    def nxsrc(self) -> int:
        return int(self.xshape.shape[0])

    @property
    def npsrc(self) -> int:
        return self.nsrc - self.ngsrc - self.nxsrc

    def params(self) -> np.ndarray:
        """[nsrc][10] parameter table (l, m, I, Q, U, V, alpha, el, em, R)."""
        out = np.zeros((self.nsrc, 10))
        out[:, 0:2] = self.lm
        out[:, 2:6] = self.stokes
        out[:, 6] = self.alpha
        n0 = self.npsrc
        if self.ngsrc:
            out[n0:n0 + self.ngsrc, 7:10] = self.gshape
        if self.nxsrc:
            out[n0 + self.ngsrc:, 7:10] = self.xshape
        return out

    @staticmethod
    def from_params(p: np.ndarray, ngsrc: int, nxsrc: int = 0) -> "Sky":
        p = np.asarray(p, dtype=np.float64)
        nsrc = p.shape[0]
        n0 = nsrc - ngsrc - nxsrc
        return Sky(lm=p[:, 0:2].copy(), stokes=p[:, 2:6].copy(), alpha=p[:, 6].copy(),
                   gshape=p[n0:n0 + ngsrc, 7:10].copy() if ngsrc else np.zeros((0, 3)),
                   xshape=p[n0 + ngsrc:, 7:10].copy() if nxsrc else np.zeros((0, 3)))

    def subset(self, np_keep: int, ng_keep: int, nx_keep: int = 0) -> "Sky":
        """The first np_keep point sources, first ng_keep Gaussian sources and
        first nx_keep exponential disks."""
        npnt, ng = self.npsrc, self.ngsrc
        idx = np.concatenate([np.arange(np_keep), npnt + np.arange(ng_keep),
                              npnt + ng + np.arange(nx_keep)]).astype(np.int64)
        return Sky(lm=self.lm[idx].copy(), stokes=self.stokes[idx].copy(),
                   alpha=self.alpha[idx].copy(), gshape=self.gshape[:ng_keep].copy(),
                   xshape=self.xshape[:nx_keep].copy())


def canonical_baselines(na: int) -> tuple[np.ndarray, np.ndarray]:
    """Antenna pairs p < q in row-major order (0,1), (0,2), ..., (na-2, na-1)."""
    p, q = np.triu_indices(na, k=1)
    return p.astype(np.int32), q.astype(np.int32)


def rngs(key: int, n: int = 6) -> list[np.random.Generator]:
    """Independent child generators for one configuration key."""
    ss = np.random.SeedSequence(BASE_SEED + key)
    return [np.random.default_rng(c) for c in ss.spawn(n)]


def make_uvw(na: int, ntime: int, uv_half: float, w_half: float,
             rng: np.random.Generator) -> np.ndarray:
    """Per-antenna uvw: u, v ~ U(-uv_half, uv_half), w ~ U(-w_half, w_half) at t = 0,
    then rotated about the w axis by ROT_PER_STEP rad per timestep."""
    u0 = rng.uniform(-uv_half, uv_half, na)
    v0 = rng.uniform(-uv_half, uv_half, na)
    w0 = rng.uniform(-w_half, w_half, na)
    th = ROT_PER_STEP * np.arange(ntime)[:, None]
    c, s = np.cos(th), np.sin(th)
    uvw = np.empty((ntime, na, 3))
    uvw[:, :, 0] = u0[None] * c - v0[None] * s
    uvw[:, :, 1] = u0[None] * s + v0[None] * c
    uvw[:, :, 2] = w0[None]
    return uvw


def make_sky(npsrc: int, ngsrc: int, rng: np.random.Generator) -> Sky:
    """Sources: l, m ~ U(-0.02, 0.02); I ~ LogNormal(0, 1); Q, U, V = I * U(-0.1, 0.1);
    alpha ~ N(-0.7, 0.2).  Gaussians: axes ~ U(1, 30) arcsec (sorted so that
    major >= minor), position angle ~ U(0, pi)."""
    n = npsrc + ngsrc
    lm = rng.uniform(-0.02, 0.02, (n, 2))
    stokes = np.empty((n, 4))
    stokes[:, 0] = rng.lognormal(0.0, 1.0, n)
    stokes[:, 1:4] = stokes[:, :1] * rng.uniform(-0.1, 0.1, (n, 3))
    alpha = rng.normal(-0.7, 0.2, n)
    ax = rng.uniform(1.0, 30.0, (ngsrc, 2)) * ARCSEC
    tmaj = ax.max(axis=1)
    tmin = ax.min(axis=1)
    pa = rng.uniform(0.0, math.pi, ngsrc)
    gshape = np.stack([tmaj * np.sin(pa), tmaj * np.cos(pa), tmin / tmaj], axis=1) \
        if ngsrc else np.zeros((0, 3))
    return Sky(lm=lm, stokes=stokes, alpha=alpha, gshape=gshape)


def add_disks(sky: Sky, nxsrc: int, rng: np.random.Generator) -> Sky:
    """`sky` followed by nxsrc exponential disks: positions, Stokes and
    spectral indices drawn as in make_sky; major-axis scale length
    h ~ U(0.5, 15) arcsec, axis ratio R ~ U(0.1, 1), position angle
    ~ U(0, pi); xshape = (h sin(pa), h cos(pa), R)."""
    extra = make_sky(nxsrc, 0, rng)
    h = rng.uniform(0.5, 15.0, nxsrc) * ARCSEC
    R = rng.uniform(0.1, 1.0, nxsrc)
    pa = rng.uniform(0.0, math.pi, nxsrc)
    xshape = np.stack([h * np.sin(pa), h * np.cos(pa), R], axis=1) if nxsrc else np.zeros((0, 3))
    return Sky(lm=np.concatenate([sky.lm, extra.lm]),
               stokes=np.concatenate([sky.stokes, extra.stokes]),
               alpha=np.concatenate([sky.alpha, extra.alpha]),
               gshape=sky.gshape, xshape=np.concatenate([sky.xshape, xshape]))


def random_die(ntime: int, na: int, nchan: int, rng: np.random.Generator,
               scale: float = 0.1) -> np.ndarray:
    """A direction-independent 2x2 complex term per (timestep, antenna,
    channel), [ntime][na][nchan][2][2]: the identity plus complex Gaussian
    entries of standard deviation `scale` in real and imaginary parts."""
    shp = (ntime, na, nchan, 2, 2)
    return np.eye(2)[None, None, None] + scale * (rng.standard_normal(shp)
                                                   + 1j * rng.standard_normal(shp))


def stokes_per_time(sky: Sky, ntime: int, rng: np.random.Generator,
                    frac: float = 0.1) -> np.ndarray:
    """Brightness per timestep, [ntime][nsrc][4]: the sky's Stokes vector
    times (1 + frac N(0, 1)) drawn per timestep, source and parameter."""
    return sky.stokes[None] * (1.0 + frac * rng.standard_normal((ntime, sky.nsrc, 4)))


def perturb(sky: Sky, rng: np.random.Generator, frac: float = PERTURB_FRAC) -> Sky:
    """Every scalar parameter multiplied by (1 + frac * N(0, 1))."""
    p = sky.params()
    p = p * (1.0 + frac * rng.standard_normal(p.shape))
    return Sky.from_params(p, sky.ngsrc, sky.nxsrc)


def make_observation(cfg: dict, rng_uvw: np.random.Generator,
                     rng_inst: np.random.Generator) -> Observation:
    na, ntime, nchan = cfg["na"], cfg["ntime"], cfg["nchan"]
    ant1, ant2 = canonical_baselines(na)
    uvw = make_uvw(na, ntime, cfg["uv_half"], cfg["w_half"], rng_uvw)
    freq = np.linspace(cfg["f0"], cfg["f1"], nchan)
    obs = Observation(ntime=ntime, na=na, nchan=nchan, ant1=ant1, ant2=ant2, uvw=uvw,
                      freq=freq, beam=bool(cfg["beam"]))
    if obs.beam:
        # pointing errors ~ N(0, 1e-4) rad per (t, antenna, axis)
        obs.pointing = rng_inst.normal(0.0, 1e-4, (ntime, na, 2))
        # gains: (1 + 0.05 N(0,1)) exp(i N(0, 0.1)) per antenna and feed
        amp = 1.0 + 0.05 * rng_inst.standard_normal((na, 2))
        ph = rng_inst.normal(0.0, 0.1, (na, 2))
        obs.gains = amp * np.exp(1j * ph)
    return obs


def noise(shape, rng: np.random.Generator, sigma: float = NOISE_SIGMA) -> np.ndarray:
    """Complex Gaussian noise: real and imaginary parts each N(0, sigma^2)."""
    return rng.normal(0.0, sigma, shape) + 1j * rng.normal(0.0, sigma, shape)


def weights(obs: Observation, sigma: float = NOISE_SIGMA) -> np.ndarray:
    return np.full((obs.ntime, obs.nbl, obs.nchan, 4), 1.0 / sigma ** 2)


@dataclass
class Problem:
    """One configuration: observation, evaluation sky, truth sky, noise and weights.

    ``data`` must be filled by the caller as model(truth) + noise."""
    name: str
    obs: Observation
    sky: Sky
    truth: Sky
    noise: np.ndarray
    weight: np.ndarray


def make_problem(name: str, *, ntime: int | None = None, nchan: int | None = None,
                 na: int | None = None, npsrc: int | None = None,
                 ngsrc: int | None = None, key: int | None = None,
                 dense: bool = True) -> Problem:
    """Build configuration ``name`` (c0 ... c4).  Optional overrides shrink it
    (the recipe and seeds are unchanged, so e.g. ``ntime`` gives a time prefix
    of the same uvw track when only ntime changes).  With dense=False the
    per-visibility noise and weight arrays are not drawn (None): for callers
    that only need the observation and the skies of a large configuration."""
    cfg = dict(CONFIGS[name])
    for k, v in (("ntime", ntime), ("nchan", nchan), ("na", na), ("npsrc", npsrc),
                 ("ngsrc", ngsrc)):
        if v is not None:
            cfg[k] = v
    if key is None:
        key = int(name[1:])
    r_uvw, r_sky, r_pert, r_noise, r_inst, _ = rngs(key)
    obs = make_observation(cfg, r_uvw, r_inst)
    sky = make_sky(cfg["npsrc"], cfg["ngsrc"], r_sky)
    truth = perturb(sky, r_pert)
    if not dense:
        return Problem(name=name, obs=obs, sky=sky, truth=truth, noise=None, weight=None)
    nz = noise((obs.ntime, obs.nbl, obs.nchan, 4), r_noise)
    return Problem(name=name, obs=obs, sky=sky, truth=truth, noise=nz, weight=weights(obs))


@dataclass
class BatchProblem:
    """Batched proposals over one shared observation (configuration c3)."""
    obs: Observation
    truth: Sky
    skies: list
    noise: np.ndarray
    weight: np.ndarray


def make_batch_problem(*, nset: int | None = None, ntime: int | None = None,
                       nchan: int | None = None, nmax: int | None = None,
                       nmin: int | None = None, key: int = 3) -> BatchProblem:
    """A truth sky of npsrc + ngsrc sources; proposal b keeps the first
    ceil((1-gfrac) n_b) point and floor(gfrac n_b) Gaussian truth sources,
    n_b ~ U{nmin..nmax}, each parameter perturbed by 1%."""
    cfg = dict(CONFIGS["c3"])
    for k, v in (("nset", nset), ("ntime", ntime), ("nchan", nchan), ("nmax", nmax),
                 ("nmin", nmin)):
        if v is not None:
            cfg[k] = v
    r_uvw, r_sky, r_pert, r_noise, r_inst, r_cnt = rngs(key)
    obs = make_observation(cfg, r_uvw, r_inst)
    truth = make_sky(cfg["npsrc"], cfg["ngsrc"], r_sky)
    counts = r_cnt.integers(cfg["nmin"], cfg["nmax"] + 1, cfg["nset"])
    skies = []
    for nb in counts:
        ng = int(math.floor(cfg["gfrac"] * nb))
        npt = int(nb) - ng
        npt = min(npt, truth.npsrc)
        ng = min(ng, truth.ngsrc)
        skies.append(perturb(truth.subset(npt, ng), r_pert))
    nz = noise((obs.ntime, obs.nbl, obs.nchan, 4), r_noise)
    return BatchProblem(obs=obs, truth=truth, skies=skies, noise=nz, weight=weights(obs))
