"""CPU oracle for the RIME chi-squared engine -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product path (the HIP library and its binding) never
does; the two share no code.

What it computes (Perkins et al. 2015, "Montblanc", Section 2.1 "The Radio
Interferometry Measurement Equation" and Section 2.3 "Bayesian Inference for
Radio Observations"), written as the plain direct sum in float64 /
complex128 torch CPU tensors:

    V_tpq(nu) = sum_s  S_tpqs(nu) * A_tps(nu) B_s(nu) A_tqs(nu)^H          (eq. 1)
    A_tps     = E_tps K_tps,  E_tps = e_tps diag(g_p0, g_p1)                (eq. e_term)
    K_tps     = exp(-2 pi i (u l + v m + w (n - 1)) nu / c)                 (eq. k_term)
    B_s       = (nu / nu_ref)^alpha [[I+Q, U+iV], [U-iV, I-Q]]              (eq. brightness_term)
    chi^2     = sum_{t,pq,nu,corr} w |V - D|^2                              (eq. lhood)

Readings taken where the paper is silent or garbled (each repeated at the
function that uses it):

* K carries a minus sign in the exponent (the paper's eq. k_term prints +; all
  invariants hold under either sign).
* The beam is e = cos^3(min(beam_k * r * nu / beam_ref_freq, beam_clip)),
  r = |(l, m) - (dl, dm)_tp|, times a diagonal complex gain per antenna; the
  paper's "C = 65 GHz times lambda" is dimensionally inconsistent.
* The Gaussian shape factor is the normalised Fourier transform of an
  elliptical Gaussian with FWHM major axis theta_maj, minor axis theta_min and
  position angle pa measured from +m towards +l, parameterised as
  el = theta_maj sin(pa), em = theta_maj cos(pa), R = theta_min / theta_maj:
      S = exp(-(pi^2 / (4 ln 2)) [(u' el + v' em)^2 + R^2 (u' em - v' el)^2]),
  u' = (u_p - u_q) nu / c, v' = (v_p - v_q) nu / c.  The paper gives no
  formula (Table rime_input only lists the parameters).
* (V - D)^2 on complex numbers is |V - D|^2, summed over the four
  correlations xx, xy, yx, yy, each with its own real weight.

* The direction-independent term G of eq. 1 (optional, a full 2x2 complex
  matrix per timestep, antenna and channel) multiplies the source sum from
  both sides: V_pq = G_p X_pq G_q^H.
* A third morphology after points and Gaussians: the elliptical exponential
  disk (Sersic index 1), parameterised like the Gaussian with the major-axis
  scale length h in place of the FWHM (disk_shape).
* Brightness may be given per timestep (Table rime_input lists an
  ntime x nsrc brightness array); the spectral index stays per source.

Gradients with respect to (l, m, I, Q, U, V, alpha, el, em, R), to G and to
the per-timestep brightness come from torch.autograd applied to the same
direct sum.  ``brute_force_vis`` restates eq. 1 with scalar Python loops for
tiny problems.

Inputs are the dataclasses of ``rime_synth`` (plain numpy arrays).
"""
from __future__ import annotations

import cmath
import math

import numpy as np
import torch

C_LIGHT = 299792458.0  # m/s, exact
GAUSS_K = math.pi ** 2 / (4.0 * math.log(2.0))

_F64 = torch.float64
_C128 = torch.complex128


def _t(x, dtype=_F64):
    return torch.as_tensor(np.asarray(x), dtype=dtype)


# --------------------------------------------------------------------------- #
# Per-term factors
# --------------------------------------------------------------------------- #

def n_minus_one(l, m):
    """n - 1 with n = sqrt(1 - l^2 - m^2) (Section 2.1, after eq. k_term),
    written as -(l^2 + m^2) / (1 + n), which is the same number without the
    cancellation of sqrt(...) - 1 near the phase centre.  Directions with
    l^2 + m^2 >= 1 lie outside the domain of n and raise ValueError."""
    r2 = l * l + m * m
    if bool((r2.detach() >= 1.0).any()):
        raise ValueError("source direction outside the domain l^2 + m^2 < 1")
    return -r2 / (1.0 + torch.sqrt(1.0 - r2))


# Error-free transformations (float64 arithmetic only, no fused multiply-add):
# they carry the phase of eq. k_term without rounding (reading R12).

def _split(a):
    """Veltkamp's split a = hi + lo, hi with at most 26 significant bits, so
    that every product of two halves is exact in float64."""
    c = 134217729.0 * a  # 2^27 + 1
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    """Dekker's product: (p, e) with p = fl(a b) and p + e = a b exactly."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def _two_sum(a, b):
    """Knuth's sum: (s, e) with s = fl(a + b) and s + e = a + b exactly."""
    s = a + b
    bv = s - a
    e = (a - (s - bv)) + (b - bv)
    return s, e


def phase_turns(uvw, lm, freq):
    """The phase of eq. k_term in turns, x = (u l + v m + w (n - 1)) nu / c
    (1/lambda = nu/c), with its integer part removed (exp(-2 pi i x) has
    period 1 in x): shape [T][A][S][F], values in [-1/2, 1/2] up to rounding.

    x reaches hundreds to thousands of turns on the benchmark arrays, so the
    path length tau and its product with nu / c are carried as float64 pairs
    (hi + lo) through error-free sums and products; the fraction is then the
    exact fraction of the products of the float64 inputs to about 1e-16
    turns (reading R12)."""
    l, m = lm[:, 0], lm[:, 1]
    nm1 = n_minus_one(l, m)
    u, v, w = uvw[..., 0][..., None], uvw[..., 1][..., None], uvw[..., 2][..., None]
    p1, e1 = _two_prod(u, l)                                          # [T][A][S]
    p2, e2 = _two_prod(v, m)
    p3, e3 = _two_prod(w, nm1)
    s, es1 = _two_sum(p1, p2)
    s, es2 = _two_sum(s, p3)
    th, tl = _two_sum(s, (e1 + e2 + e3) + (es1 + es2))               # tau = th + tl
    nuc = freq / C_LIGHT                                               # [F]
    xh, xe = _two_prod(th[..., None], nuc)                             # [T][A][S][F]
    xl = xe + tl[..., None] * nuc
    return (xh - torch.round(xh)) + xl


def phase_K(uvw, lm, freq):
    """K_tps = exp(-2 pi i x), x = phase_turns (eq. k_term, sign reading '-');
    the angle passed to exp stays within [-pi, pi]."""
    frac = phase_turns(uvw, lm, freq)
    return torch.exp(torch.complex(torch.zeros_like(frac), -2.0 * math.pi * frac))


def beam_e(lm, pointing, freq, k, ref_freq, clip):
    """Real cos^3 beam factor e_tps(nu), shape [T][A][S][F] (eq. e_term, read
    as cos^3(min(k * r * nu / ref_freq, clip)) with r the distance of the
    source from the antenna's pointing centre)."""
    dl = lm[None, None, :, 0] - pointing[..., 0][..., None]
    dm = lm[None, None, :, 1] - pointing[..., 1][..., None]
    # r = |(dl, dm)|; at r = 0 (a source on the pointing centre) e is smooth
    # with zero derivative, which the square root's infinite slope would turn
    # into NaN under autograd: the derivative there is taken as its limit, 0
    r2 = dl * dl + dm * dm
    on = r2 > 0
    r = torch.sqrt(torch.where(on, r2, torch.ones_like(r2))) * on       # [T][A][S]
    arg = torch.clamp(k * r[..., None] * (freq / ref_freq), max=clip)  # [T][A][S][F]
    return torch.cos(arg) ** 3


def spectral(alpha, freq, ref_freq):
    """(lambda_ref / lambda)^alpha = (nu / nu_ref)^alpha, shape [S][F]
    (eq. brightness_term)."""
    return torch.pow((freq / ref_freq)[None, :], alpha[:, None])


def brightness(stokes, alpha, freq, ref_freq):
    """B_s(nu) = (nu/nu_ref)^alpha [[I+Q, U+iV], [U-iV, I-Q]], shape
    [S][F][2][2] (eq. brightness_term; no factor 1/2, as printed)."""
    I, Q, U, V = stokes[:, 0], stokes[:, 1], stokes[:, 2], stokes[:, 3]
    zero = torch.zeros_like(I)
    b = torch.stack([
        torch.stack([torch.complex(I + Q, zero), torch.complex(U, V)], dim=-1),
        torch.stack([torch.complex(U, -V), torch.complex(I - Q, zero)], dim=-1),
    ], dim=-2)                                                            # [S][2][2]
    f = spectral(alpha, freq, ref_freq)                                   # [S][F]
    return b[:, None] * f[..., None, None].to(_C128)


def gauss_shape(duvw, gshape, freq):
    """Gaussian shape factor S_tpqs(nu), shape [T][B][G][F] (reading in the
    module docstring).  duvw = uvw_p - uvw_q per baseline, [T][B][3]; the w
    component does not enter."""
    el, em, R = gshape[:, 0], gshape[:, 1], gshape[:, 2]
    s = freq / C_LIGHT
    up = duvw[..., 0][..., None, None] * s            # [T][B][1][F]
    vp = duvw[..., 1][..., None, None] * s
    el_, em_, R_ = el[:, None], em[:, None], R[:, None]
    a = up * el_ + vp * em_
    b = up * em_ - vp * el_
    return torch.exp(-GAUSS_K * (a * a + R_ * R_ * b * b))


def disk_shape(duvw, xshape, freq):
    """Shape factor of an elliptical exponential disk (a Sersic profile of
    index 1), shape [T][B][X][F].  The sky-plane profile is
    exp(-sqrt((x / h)^2 + (y / (R h))^2)) with scale length h (rad) along the
    major axis x at position angle pa (from +m towards +l) and axis ratio R;
    parameters (el, em, R) = (h sin pa, h cos pa, R) as for the Gaussian.  Its
    normalised 2-D Fourier transform at baseline (u', v') = (u_p - u_q,
    v_p - v_q) nu / c is
        S = (1 + (2 pi)^2 [(u' el + v' em)^2 + R^2 (u' em - v' el)^2])^(-3/2)
    (the circular case is the textbook transform of exp(-r/h),
    2 pi h^2 (1 + (2 pi h k)^2)^(-3/2); the ellipse stretches k along the
    axes).  The w component does not enter."""
    el, em, R = xshape[:, 0], xshape[:, 1], xshape[:, 2]
    s = freq / C_LIGHT
    up = duvw[..., 0][..., None, None] * s            # [T][B][1][F]
    vp = duvw[..., 1][..., None, None] * s
    el_, em_, R_ = el[:, None], em[:, None], R[:, None]
    a = up * el_ + vp * em_
    b = up * em_ - vp * el_
    return (1.0 + (2.0 * math.pi) ** 2 * (a * a + R_ * R_ * b * b)) ** -1.5


def jones_A(obs_t, lm, freq):
    """Per-antenna A = E K as full 2x2 matrices, [T][A][S][F][2][2]."""
    uvw, pointing, gains = obs_t["uvw"], obs_t["pointing"], obs_t["gains"]
    K = phase_K(uvw, lm, freq)                                           # [T][A][S][F]
    T, A, S, F = K.shape
    if obs_t["beam"]:
        e = beam_e(lm, pointing, freq, obs_t["beam_k"], obs_t["beam_ref_freq"],
                   obs_t["beam_clip"]).to(_C128)
        scal = e * K
    else:
        scal = K
    g = gains if gains is not None else torch.ones((A, 2), dtype=_C128)
    Emat = torch.zeros((A, 2, 2), dtype=_C128)
    Emat[:, 0, 0] = g[:, 0]
    Emat[:, 1, 1] = g[:, 1]
    return scal[..., None, None] * Emat[None, :, None, None]             # [T][A][S][F][2][2]


# --------------------------------------------------------------------------- #
# Visibilities and chi-squared
# --------------------------------------------------------------------------- #

def _obs_tensors(obs, t0, t1):
    d = {
        "uvw": _t(obs.uvw[t0:t1]),
        "beam": bool(obs.beam),
        "pointing": _t(obs.pointing[t0:t1]) if obs.pointing is not None
        else torch.zeros((t1 - t0, obs.na, 2), dtype=_F64),
        "gains": _t(obs.gains, _C128) if obs.gains is not None else None,
        "beam_k": float(obs.beam_k),
        "beam_ref_freq": float(obs.beam_ref_freq),
        "beam_clip": float(obs.beam_clip),
    }
    return d


def _vis_block(obs, t0, t1, lm, stokes, alpha, gshape, ngsrc, src_chunk, xshape=None,
               nxsrc=0):
    """Source-summed coherency for timesteps [t0, t1): [T][B][F][2][2]
    complex128.  Sources are points, then ngsrc Gaussians (gshape), then
    nxsrc exponential disks (xshape); stokes is [S][4]."""
    freq = _t(obs.freq)
    ant1 = torch.as_tensor(np.asarray(obs.ant1, dtype=np.int64))
    ant2 = torch.as_tensor(np.asarray(obs.ant2, dtype=np.int64))
    ot = _obs_tensors(obs, t0, t1)
    nsrc = lm.shape[0]
    npsrc = nsrc - ngsrc - nxsrc
    nx0 = npsrc + ngsrc                                                  # first disk
    T, Bn, F = t1 - t0, ant1.shape[0], freq.shape[0]
    duvw = ot["uvw"][:, ant1] - ot["uvw"][:, ant2]                       # [T][B][3]
    vis = torch.zeros((T, Bn, F, 2, 2), dtype=_C128)
    for s0 in range(0, nsrc, src_chunk):
        s1 = min(nsrc, s0 + src_chunk)
        A = jones_A(ot, lm[s0:s1], freq)                                 # [T][A][s][F][2][2]
        Bm = brightness(stokes[s0:s1], alpha[s0:s1], freq, obs.ref_freq)  # [s][F][2][2]
        Ap = A[:, ant1]                                                  # [T][B][s][F][2][2]
        Aq = A[:, ant2]
        X = Ap @ Bm[None, None] @ Aq.conj().transpose(-1, -2)            # source coherency
        parts = []
        if min(s1, npsrc) > s0:                                          # points: S = 1
            parts.append(torch.ones((T, Bn, min(s1, npsrc) - s0, F), dtype=_F64))
        g0, g1 = max(s0, npsrc), min(s1, nx0)
        if g1 > g0:
            parts.append(gauss_shape(duvw, gshape[g0 - npsrc:g1 - npsrc], freq))
        x0, x1 = max(s0, nx0), s1
        if x1 > x0:
            parts.append(disk_shape(duvw, xshape[x0 - nx0:x1 - nx0], freq))
        if s1 > npsrc:
            X = X * torch.cat(parts, dim=2)[..., None, None].to(_C128)
        vis = vis + X.sum(dim=2)
    return vis


def apply_die(vis, G, ant1, ant2):
    """V_tpq(nu) = G_tp(nu) X_tpq(nu) G_tq(nu)^H: the direction-independent
    2x2 term of eq. 1, applied outside the source sum.  vis [T][B][F][2][2],
    G [T][A][F][2][2] complex."""
    a1 = torch.as_tensor(np.asarray(ant1, dtype=np.int64))
    a2 = torch.as_tensor(np.asarray(ant2, dtype=np.int64))
    Gp = G[:, a1]
    Gq = G[:, a2]
    return Gp @ vis @ Gq.conj().transpose(-1, -2)


def _sky_tensors(sky):
    xs = getattr(sky, "xshape", None)
    return (_t(sky.lm), _t(sky.stokes), _t(sky.alpha), _t(sky.gshape),
            _t(xs) if xs is not None else torch.zeros((0, 3), dtype=_F64))


def model_vis(obs, sky, src_chunk: int = 64, die=None, stokes_t=None):
    """Model visibilities V_tpq(nu) as [T][B][F][4] complex128 numpy, correlations
    ordered xx, xy, yx, yy (eq. 1 with the source coherency and its sum).
    die: optional [T][A][F][2][2] complex direction-independent term;
    stokes_t: optional [T][S][4] brightness per timestep (replaces
    sky.stokes; Table rime_input gives the brightness per timestep)."""
    lm, stokes, alpha, gshape, xshape = _sky_tensors(sky)
    nx = getattr(sky, "nxsrc", 0)
    out = np.empty((obs.ntime, obs.nbl, obs.nchan, 4), dtype=np.complex128)
    for t in range(obs.ntime):
        st = _t(stokes_t[t]) if stokes_t is not None else stokes
        v = _vis_block(obs, t, t + 1, lm, st, alpha, gshape, sky.ngsrc, src_chunk, xshape, nx)
        if die is not None:
            v = apply_die(v, _t(die[t:t + 1], _C128), obs.ant1, obs.ant2)
        out[t] = v.reshape(obs.nbl, obs.nchan, 4).numpy()
    return out


def chi2_from_vis(vis, data, weight) -> float:
    """chi^2 = sum w |V - D|^2 (eq. lhood; the ln(2 pi / w) constant excluded)."""
    r = np.asarray(vis) - np.asarray(data)
    return float(np.sum(np.asarray(weight) * (r.real ** 2 + r.imag ** 2)))


def loglike_const(weight) -> float:
    """sum ln(2 pi / w), the weight-only term of -2 ln L (eq. lhood)."""
    return float(np.sum(np.log(2.0 * math.pi / np.asarray(weight, dtype=np.float64))))


def chi2(obs, sky, data, weight, src_chunk: int = 64) -> float:
    """chi^2 of the model for ``sky`` against ``data`` (eq. lhood)."""
    return chi2_from_vis(model_vis(obs, sky, src_chunk), data, weight)


def chi2_and_grad(obs, sky, data, weight, src_chunk: int = 64, t_chunk: int = 1):
    """(chi^2, grad) with grad[s] = d chi^2 / d(l, m, I, Q, U, V, alpha, el, em, R)
    for every source (shape columns zero for point sources), by autograd of the
    direct sum, accumulated over time chunks (chi^2 is additive over time)."""
    r = chi2_and_grad_ext(obs, sky, data, weight, src_chunk=src_chunk, t_chunk=t_chunk)
    return r["chi2"], r["grad"]


def chi2_and_grad_ext(obs, sky, data, weight, die=None, stokes_t=None, src_chunk: int = 64,
                      t_chunk: int = 1):
    """chi^2 and its gradients by autograd of the direct sum, with the optional
    direction-independent term `die` [T][A][F][2][2] complex and brightness
    per timestep `stokes_t` [T][S][4].  Returns a dict:
      chi2;
      grad [S][10]: d chi^2 / d(l, m, I, Q, U, V, alpha, shape) (with stokes_t,
        the Stokes columns are d chi^2 / d(a common offset of all timesteps),
        i.e. the sum over t of grad_stokes_t);
      grad_die [T][A][F][2][2] complex: d chi^2 / d Re G + i d chi^2 / d Im G;
      grad_stokes_t [T][S][4]."""
    lm, stokes, alpha, gshape, xshape = _sky_tensors(sky)
    for x in (lm, stokes, alpha, gshape, xshape):
        x.requires_grad_(True)
    nx = getattr(sky, "nxsrc", 0)
    G = _t(die, _C128).requires_grad_(True) if die is not None else None
    St = _t(stokes_t).requires_grad_(True) if stokes_t is not None else None
    if St is not None:
        t_chunk = 1
    D = np.asarray(data)
    W = np.asarray(weight, dtype=np.float64)
    total = 0.0
    for t0 in range(0, obs.ntime, t_chunk):
        t1 = min(obs.ntime, t0 + t_chunk)
        st = St[t0] if St is not None else stokes
        v = _vis_block(obs, t0, t1, lm, st, alpha, gshape, sky.ngsrc, src_chunk, xshape, nx)
        if G is not None:
            v = apply_die(v, G[t0:t1], obs.ant1, obs.ant2)
        v = v.reshape(t1 - t0, obs.nbl, obs.nchan, 4)
        r = v - torch.as_tensor(D[t0:t1], dtype=_C128)
        c = (torch.as_tensor(W[t0:t1]) * (r.real ** 2 + r.imag ** 2)).sum()
        c.backward()
        total += float(c.detach())
    g = np.zeros((sky.nsrc, 10))
    g[:, 0:2] = lm.grad.numpy()
    g[:, 6] = alpha.grad.numpy()
    npsrc = sky.nsrc - sky.ngsrc - nx
    if sky.ngsrc:
        g[npsrc:npsrc + sky.ngsrc, 7:10] = gshape.grad.numpy()
    if nx:
        g[npsrc + sky.ngsrc:, 7:10] = xshape.grad.numpy()
    out = {"chi2": total, "grad": g}
    if St is not None:
        out["grad_stokes_t"] = St.grad.numpy()
        g[:, 2:6] = St.grad.numpy().sum(axis=0)
    else:
        g[:, 2:6] = stokes.grad.numpy()
    if G is not None:
        out["grad_die"] = G.grad.numpy()
    return out


# --------------------------------------------------------------------------- #
# Brute force: eq. 1 with scalar loops (tiny problems only)
# --------------------------------------------------------------------------- #

def _mm(a, b):
    return [[a[0][0] * b[0][0] + a[0][1] * b[1][0], a[0][0] * b[0][1] + a[0][1] * b[1][1]],
            [a[1][0] * b[0][0] + a[1][1] * b[1][0], a[1][0] * b[0][1] + a[1][1] * b[1][1]]]


def _herm(a):
    return [[a[0][0].conjugate(), a[1][0].conjugate()],
            [a[0][1].conjugate(), a[1][1].conjugate()]]


def brute_force_vis(obs, sky):
    """V_tpq(nu) from eq. 1 with explicit scalar loops over t, baselines,
    channels and sources and explicit 2x2 Jones products E K B K^H E^H.
    Returns [T][B][F][4] complex numpy."""
    out = np.zeros((obs.ntime, obs.nbl, obs.nchan, 4), dtype=np.complex128)
    npsrc = sky.npsrc
    for t in range(obs.ntime):
        for b in range(obs.nbl):
            p, q = int(obs.ant1[b]), int(obs.ant2[b])
            for f, nu in enumerate(obs.freq):
                lam = C_LIGHT / nu
                acc = [[0j, 0j], [0j, 0j]]
                for s in range(sky.nsrc):
                    l, m = sky.lm[s]
                    n = math.sqrt(1.0 - l * l - m * m)
                    I, Q, U, V = sky.stokes[s]
                    spec = (nu / obs.ref_freq) ** sky.alpha[s]
                    Bm = [[spec * (I + Q), spec * complex(U, V)],
                          [spec * complex(U, -V), spec * (I - Q)]]
                    jones = []
                    for a in (p, q):
                        u, v, w = obs.uvw[t, a]
                        k = cmath.exp(-2j * math.pi * (u * l + v * m + w * (n - 1.0)) / lam)
                        if obs.beam:
                            dl = l - obs.pointing[t, a, 0]
                            dm = m - obs.pointing[t, a, 1]
                            r = math.sqrt(dl * dl + dm * dm)
                            e = math.cos(min(obs.beam_k * r * nu / obs.beam_ref_freq,
                                             obs.beam_clip)) ** 3
                        else:
                            e = 1.0
                        g = obs.gains[a] if obs.gains is not None else (1.0, 1.0)
                        jones.append([[e * k * g[0], 0j], [0j, e * k * g[1]]])
                    X = _mm(_mm(jones[0], Bm), _herm(jones[1]))
                    if s >= npsrc:
                        el, em, R = sky.gshape[s - npsrc]
                        du = (obs.uvw[t, p, 0] - obs.uvw[t, q, 0]) / lam
                        dv = (obs.uvw[t, p, 1] - obs.uvw[t, q, 1]) / lam
                        sh = math.exp(-GAUSS_K * ((du * el + dv * em) ** 2
                                                  + (R * (du * em - dv * el)) ** 2))
                    else:
                        sh = 1.0
                    for i in range(2):
                        for j in range(2):
                            acc[i][j] += sh * X[i][j]
                out[t, b, f] = [acc[0][0], acc[0][1], acc[1][0], acc[1][1]]
    return out


def total_flux(sky, freq, ref_freq):
    """F(nu) = sum_s I_s (nu/nu_ref)^alpha_s, per channel: the scale against
    which visibility errors are judged."""
    f = np.power(np.asarray(freq)[None, :] / ref_freq, np.asarray(sky.alpha)[:, None])
    return (np.asarray(sky.stokes)[:, 0:1] * f).sum(axis=0)
