"""Shared helpers for the GPU parity tests: problem construction (inputs from
rime_synth, observed data from the oracle) and the error metrics."""
from __future__ import annotations

import numpy as np

import oracle.rime_oracle as O
from rime_synth import make_problem

# Tolerances against the oracle: FP64 path, float32-mixed path, and the mixed
# path with a float64 forward (float64 residual, float32 adjoint).
TOL = {0: 1e-12, 1: 1e-5, 2: 1e-5}


def round_inputs(D, W, prec):
    """The mixed precisions consume complex64/float32 data; the oracle gets
    the same rounded values so parity measures compute error only."""
    if prec != 0:
        return (D.astype(np.complex64).astype(np.complex128),
                W.astype(np.float32).astype(np.float64))
    return D, W


def small_problem(name="c1", ntime=2, nchan=8, npsrc=40, ngsrc=20, na=None, key=None):
    pr = make_problem(name, ntime=ntime, nchan=nchan, npsrc=npsrc, ngsrc=ngsrc, na=na, key=key)
    D = O.model_vis(pr.obs, pr.truth) + pr.noise
    return pr, D, pr.weight


def vis_error(V, Vref, sky, obs):
    """max over (t, baseline, corr) of |dV| / F_nu, maximised over channels."""
    F = O.total_flux(sky, obs.freq, obs.ref_freq)          # [nchan]
    err = np.abs(np.asarray(V) - np.asarray(Vref)).max(axis=(0, 1, 3))
    return float((err / F).max())


def rel(a, b):
    return abs(a - b) / abs(b)


def grad_errors(g, gref, npsrc):
    """Per parameter type: ||dg||_2 / ||g||_2 (shape columns over Gaussians only)."""
    out = {}
    names = ["l", "m", "I", "Q", "U", "V", "alpha", "el", "em", "R"]
    for k, nm in enumerate(names):
        rows = slice(npsrc, None) if k >= 7 else slice(None)
        a, b = np.asarray(g)[rows, k], np.asarray(gref)[rows, k]
        if b.size == 0:
            continue
        nb = np.linalg.norm(b)
        out[nm] = float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
    return out


def grad_component_errors(g, gref, npsrc, floor="max"):
    """Per parameter type: the largest |dg_i| / max(|g_i|, f) with the floor
    f = 1e-3 max_type |g| (floor="max") or f = the root mean square of the
    type (floor="rms")."""
    g, gref = np.asarray(g), np.asarray(gref)
    out = {}
    names = ["l", "m", "I", "Q", "U", "V", "alpha", "el", "em", "R"]
    for k, nm in enumerate(names):
        rows = slice(npsrc, None) if k >= 7 else slice(None)
        a, b = g[rows, k], gref[rows, k]
        if b.size == 0:
            continue
        f = 1e-3 * np.abs(b).max() if floor == "max" else np.sqrt(np.mean(b * b))
        if f == 0:
            continue
        out[nm] = float((np.abs(a - b) / np.maximum(np.abs(b), f)).max())
    return out


def grad_component_worst(g, gref, npsrc):
    """Largest |dg_i| / max(|g_i|, 1e-3 * max_type |g|) over all components."""
    return max(grad_component_errors(g, gref, npsrc).values(), default=0.0)


def contribution_scale(obs, sky, D, W):
    """Per (source, parameter): sum over visibilities of |d(w |V - D|^2)/d theta|,
    by central differences of the oracle's per-visibility terms.  A summation
    error bound scales with this, not with the (possibly cancelling) sum."""
    from rime_synth import Sky
    p0 = sky.params()
    out = np.zeros_like(p0)
    for s in range(sky.nsrc):
        for k in range(10):
            if k >= 7 and s < sky.npsrc:
                continue
            h = 1e-6 * max(abs(p0[s, k]), 1e-3)
            pp, pm = p0.copy(), p0.copy()
            pp[s, k] += h
            pm[s, k] -= h
            tp = W * np.abs(O.model_vis(obs, Sky.from_params(pp, sky.ngsrc)) - D) ** 2
            tm = W * np.abs(O.model_vis(obs, Sky.from_params(pm, sky.ngsrc)) - D) ** 2
            out[s, k] = np.abs((tp - tm) / (2 * h)).sum()
    return out
