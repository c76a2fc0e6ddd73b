"""CPU-only checks of the C ABI library: it loads, exports every symbol that
include/rime.h declares, validates arguments before any HIP call, and its
host-side baseline tiling covers every baseline exactly once."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from rime_synth import canonical_baselines

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rime.h")

R = pytest.importorskip("paper_1501_07719_amd")


@pytest.fixture(scope="module")
def lib():
    return R.load_library()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rime_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in range(7):
        assert lib.rime_status_string(s)
    assert lib.rime_status_string(0) == b"ok"


def test_loglike_const_matches_definition(lib):
    w = np.random.default_rng(0).uniform(0.5, 1e4, 1000)
    ref = sum(math.log(2 * math.pi / x) for x in w)
    assert abs(R.rime_loglike_const(w) - ref) <= 1e-12 * abs(ref)


def test_variant_table(lib):
    for mode in range(3):
        for prec in range(3):
            n = R.rime_variant_count(mode, prec)
            if prec == R.MIXED_RES64 and mode == R.MODE_PREDICT:
                assert n == 0  # no predict entry point in the float64-residual precision
                continue
            assert n >= 1
            for i in range(n):
                t, c, s = R.rime_variant_info(mode, prec, i)
                assert t in (64, 256, 1024) and c >= 1 and s >= 1
                if mode == 2:
                    assert s * c == 64  # one wavefront covers a source tile x channels
    with pytest.raises(R.RimeError):
        R.rime_variant_info(0, 0, 99)


def _obs_desc(**kw):
    d = R.rime.ObsDesc()
    d.ntime, d.na, d.nbl, d.nchan = kw.get("ntime", 2), kw.get("na", 4), kw.get("nbl", 6), kw.get(
        "nchan", 3)
    return d


def test_plan_create_rejects_bad_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.rime_plan_create(None, ctypes.byref(h)) == 1
    uvw = np.zeros((2, 4, 3))
    freq = np.array([1e9, 1.1e9, 1.2e9])
    keep = []

    def mk(**kw):
        d = _obs_desc(**kw)
        d.uvw = uvw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.freq = freq.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.ref_freq = 1.4e9
        keep.append(d)
        return d

    assert lib.rime_plan_create(ctypes.byref(mk(na=1)), ctypes.byref(h)) == 1
    assert lib.rime_plan_create(ctypes.byref(mk(ntime=0)), ctypes.byref(h)) == 1
    assert lib.rime_plan_create(ctypes.byref(mk(nchan=0)), ctypes.byref(h)) == 1
    assert lib.rime_plan_create(ctypes.byref(mk(nbl=5)), ctypes.byref(h)) == 1  # not 4*3/2
    d = mk()
    d.ref_freq = 0.0
    assert lib.rime_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    d = mk()
    bad = np.array([0, 1, 2, 3, 0, 9], np.int32)
    ok = np.array([1, 2, 3, 0, 2, 1], np.int32)
    d.ant1 = bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.ant2 = ok.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.rime_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    d = mk()
    d.beam = 2
    assert lib.rime_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    for clip in (0.0, 1.6):  # beam_clip must lie in (0, 1.5]
        d = mk()
        d.beam, d.beam_k, d.beam_ref_freq, d.beam_clip = 1, 65.0, 1.4e9, clip
        assert lib.rime_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    f2 = np.array([1e9, -1.0, 1.2e9])
    d = mk()
    d.freq = f2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.rime_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1


def test_calls_reject_null_plan(lib):
    sky = R.rime.SkyDesc()
    assert lib.rime_predict(None, ctypes.byref(sky), 0, None, None, 0, None) == 1
    assert lib.rime_chi2(None, ctypes.byref(sky), 0, None, None, None, None, 0, None) == 1
    assert lib.rime_chi2_grad(None, ctypes.byref(sky), 0, None, None, None, None, None, 0,
                              None) == 1
    assert lib.rime_batch_create(None, 1, ctypes.byref(sky), ctypes.byref(ctypes.c_void_p())) == 1
    assert lib.rime_chi2_batched(None, 0, None, None, None, None, None, 0, None, 0) == 1
    assert lib.rime_workspace_size(None, 0, 0, 1, 1) == 0


def _check_tiling(na, a1, a2, threads):
    bl, lpq, ant = R.rime_tiling_host(na, a1, a2, threads)
    nat = ant.shape[1]
    seen = np.zeros(len(a1), int)
    for t in range(bl.shape[0]):
        ants = ant[t]
        nant = int((ants >= 0).sum())
        assert np.all(ants[:nant] >= 0) and np.all(ants[nant:] == -1)
        assert len(set(ants[:nant].tolist())) == nant <= nat
        for i in range(threads):
            b = bl[t, i]
            if b < 0:
                continue
            seen[b] += 1
            lp, lq = lpq[t, i] & 0xFFFF, lpq[t, i] >> 16
            assert lp < nant and lq < nant
            assert ants[lp] == a1[b] and ants[lq] == a2[b]
        # active slots first
        act = bl[t] >= 0
        assert not np.any(act[np.argmin(act):]) if not act.all() else True
    assert np.all(seen == 1)
    return bl.shape[0]


@pytest.mark.parametrize("na", [2, 7, 17, 33, 64, 197])
@pytest.mark.parametrize("threads", [64, 256, 1024])
def test_tiling_canonical(na, threads):
    a1, a2 = canonical_baselines(na)
    nt = _check_tiling(na, a1, a2, threads)
    # efficiency: tiles are not much more numerous than the ideal count
    assert nt <= math.ceil(len(a1) / threads) * 2 + 2


def test_tiling_arbitrary_lists():
    rng = np.random.default_rng(0)
    na = 40
    a1, a2 = canonical_baselines(na)
    perm = rng.permutation(len(a1))
    a1, a2 = a1[perm].copy(), a2[perm].copy()
    sw = rng.random(len(a1)) < 0.5
    a1[sw], a2[sw] = a2[sw], a1[sw].copy()
    a1 = np.concatenate([a1, a1[:50], np.arange(5)]).astype(np.int32)  # duplicates + autocorr
    a2 = np.concatenate([a2, a2[:50], np.arange(5)]).astype(np.int32)
    for threads in (64, 256, 1024):
        _check_tiling(na, a1, a2, threads)


def test_residual_precision_variants_mirror_the_others(lib):
    """The float64-residual precision's chi^2 variants are the FP64 forwards
    and its gradient variants the float32-mixed adjoints (same shapes, same
    matrix-core flags)."""
    for i in range(R.rime_variant_count(R.MODE_CHI2, R.MIXED_RES64)):
        assert R.rime_variant_info(R.MODE_CHI2, R.MIXED_RES64, i) == \
            R.rime_variant_info(R.MODE_CHI2, R.FP64, i)
        assert not R.rime_variant_matrix_cores(R.MODE_CHI2, R.MIXED_RES64, i)
    assert R.rime_variant_count(R.MODE_CHI2_GRAD, R.MIXED_RES64) == \
        R.rime_variant_count(R.MODE_CHI2_GRAD, R.MIXED)
    for i in range(R.rime_variant_count(R.MODE_CHI2_GRAD, R.MIXED)):
        assert R.rime_variant_info(R.MODE_CHI2_GRAD, R.MIXED_RES64, i) == \
            R.rime_variant_info(R.MODE_CHI2_GRAD, R.MIXED, i)
        assert R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, R.MIXED_RES64, i) == \
            R.rime_variant_matrix_cores(R.MODE_CHI2_GRAD, R.MIXED, i)


def test_domain_status_rejects_bad_arguments(lib):
    assert lib.rime_domain_status(None, 0, None) == 1
    assert lib.rime_domain_status(None, 1024, None) == 1
