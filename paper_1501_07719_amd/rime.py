"""ctypes binding of librime.so (include/rime.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device arrays are torch CUDA tensors (used for memory and streams);
the library never sees torch types, only raw pointers.  Importing this module
does not load the library; the first call does, and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librime.so")

FP64 = 0
MIXED = 1
MIXED_RES64 = 2  # float64 forward and residual, float32 adjoint (chi^2 entry points)
MODE_PREDICT = 0
MODE_CHI2 = 1
MODE_CHI2_GRAD = 2

STATUS = {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "HIP runtime error",
          4: "unsupported request", 5: "device allocation failed",
          6: "source outside the domain l^2 + m^2 < 1"}
RIME_ERR_DOMAIN = 6

C_LIGHT = 299792458.0


class RimeError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status})")


class ObsDesc(ctypes.Structure):
    _fields_ = [
        ("ntime", ctypes.c_int32), ("na", ctypes.c_int32), ("nbl", ctypes.c_int32),
        ("nchan", ctypes.c_int32),
        ("ant1", ctypes.POINTER(ctypes.c_int32)), ("ant2", ctypes.POINTER(ctypes.c_int32)),
        ("uvw", ctypes.POINTER(ctypes.c_double)), ("freq", ctypes.POINTER(ctypes.c_double)),
        ("ref_freq", ctypes.c_double), ("beam", ctypes.c_int32),
        ("pointing", ctypes.POINTER(ctypes.c_double)), ("gains", ctypes.POINTER(ctypes.c_double)),
        ("beam_k", ctypes.c_double), ("beam_ref_freq", ctypes.c_double),
        ("beam_clip", ctypes.c_double),
    ]


class SkyDesc(ctypes.Structure):
    _fields_ = [
        ("npsrc", ctypes.c_int32), ("ngsrc", ctypes.c_int32),
        ("lm", ctypes.c_void_p), ("stokes", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
        ("gshape", ctypes.c_void_p), ("nxsrc", ctypes.c_int32), ("xshape", ctypes.c_void_p),
    ]


class TermsDesc(ctypes.Structure):
    _fields_ = [("die", ctypes.c_void_p), ("grad_die", ctypes.c_void_p),
                ("stokes_t", ctypes.c_void_p), ("grad_stokes_t", ctypes.c_void_p)]


_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load librime.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"librime.so not found at {p}: run __graft_entry__.build() first")
    # torch first, so that its HIP runtime is the one the library binds to
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    vp, i32, i64, sz, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                             ctypes.c_double)
    sig = {
        "rime_plan_create": (i32, [ctypes.POINTER(ObsDesc), ctypes.POINTER(vp)]),
        "rime_plan_destroy": (None, [vp]),
        "rime_workspace_size": (sz, [vp, i32, i32, i32, i64]),
        "rime_predict": (i32, [vp, ctypes.POINTER(SkyDesc), i32, vp, vp, sz, vp]),
        "rime_chi2": (i32, [vp, ctypes.POINTER(SkyDesc), i32, vp, vp, vp, vp, sz, vp]),
        "rime_chi2_grad": (i32, [vp, ctypes.POINTER(SkyDesc), i32, vp, vp, vp, vp, vp, sz, vp]),
        "rime_batch_create": (i32, [vp, i32, ctypes.POINTER(SkyDesc), ctypes.POINTER(vp)]),
        "rime_batch_destroy": (None, [vp]),
        "rime_chi2_batched": (i32, [vp, i32, vp, vp, vp, vp, vp, sz, vp, i32]),
        "rime_batch_workspace_size": (sz, [vp, i32, i32]),
        "rime_batch_autotune": (i32, [vp, i32, i32, vp, vp, vp, sz]),
        "rime_batch_set_variant": (i32, [vp, i32, i32, i32]),
        "rime_batch_get_variant": (i32, [vp, i32, i32]),
        "rime_loglike_const": (dbl, [ctypes.POINTER(ctypes.c_double), sz]),
        "rime_status_string": (ctypes.c_char_p, [i32]),
        "rime_domain_status": (i32, [vp, sz, vp]),
        "rime_chi2_grad_noalloc": (i32, [vp, ctypes.POINTER(SkyDesc), i32, vp, vp, vp, vp, vp]),
        "rime_workspace_size_ex": (sz, [vp, i32, i32, i64, ctypes.POINTER(TermsDesc)]),
        "rime_predict_ex": (i32, [vp, ctypes.POINTER(SkyDesc), ctypes.POINTER(TermsDesc), i32, vp,
                                  vp, sz, vp]),
        "rime_chi2_ex": (i32, [vp, ctypes.POINTER(SkyDesc), ctypes.POINTER(TermsDesc), i32, vp,
                               vp, vp, vp, vp, sz, vp]),
        "rime_streamed_workspace_size": (sz, [vp, i32, i32, i64, i32]),
        "rime_chi2_streamed": (i32, [vp, ctypes.POINTER(SkyDesc), i32, vp, vp, vp, vp, i32, vp,
                                     sz, vp]),
        "rime_last_hip_error": (i32, []),
        "rime_autotune": (i32, [vp, ctypes.POINTER(SkyDesc), i32, i32, vp, vp, vp, sz,
                                ctypes.c_char_p]),
        "rime_variant_count": (i32, [i32, i32]),
        "rime_variant_matrix_cores": (i32, [i32, i32, i32]),
        "rime_variant_info": (i32, [i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]),
        "rime_set_variant": (i32, [vp, i32, i32, i32]),
        "rime_get_variant": (i32, [vp, i32, i32]),
        "rime_plan_set_timing_events": (i32, [vp, vp, vp]),
        "rime_plan_set_main_events": (i32, [vp, vp, vp]),
        "rime_tiling_host": (i32, [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32, i32,
                                   ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        raise RimeError(status, what)


def _dptr(x) -> int:
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _f64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """rime_plan_create over an observation (any object with the attributes of
    rime_synth.Observation: ntime, na, nchan, ant1, ant2, uvw, freq, ref_freq,
    beam, pointing, gains, beam_k, beam_ref_freq, beam_clip)."""

    def __init__(self, obs):
        lib = load_library()
        self.ntime, self.na, self.nchan = int(obs.ntime), int(obs.na), int(obs.nchan)
        self.nbl = int(len(obs.ant1))
        a1 = np.ascontiguousarray(obs.ant1, dtype=np.int32)
        a2 = np.ascontiguousarray(obs.ant2, dtype=np.int32)
        uvw = np.ascontiguousarray(obs.uvw, dtype=np.float64)
        freq = np.ascontiguousarray(obs.freq, dtype=np.float64)
        d = ObsDesc()
        d.ntime, d.na, d.nbl, d.nchan = self.ntime, self.na, self.nbl, self.nchan
        d.ant1, d.ant2 = _i32p(a1), _i32p(a2)
        d.uvw, d.freq = _f64p(uvw), _f64p(freq)
        d.ref_freq = float(obs.ref_freq)
        d.beam = 1 if obs.beam else 0
        keep = [a1, a2, uvw, freq]
        if obs.beam and obs.pointing is not None:
            pnt = np.ascontiguousarray(obs.pointing, dtype=np.float64)
            keep.append(pnt)
            d.pointing = _f64p(pnt)
        if obs.gains is not None:
            g = np.ascontiguousarray(np.asarray(obs.gains, dtype=np.complex128)).view(np.float64)
            g = np.ascontiguousarray(g)
            keep.append(g)
            d.gains = _f64p(g)
        d.beam_k, d.beam_ref_freq, d.beam_clip = (float(obs.beam_k), float(obs.beam_ref_freq),
                                                  float(obs.beam_clip))
        h = ctypes.c_void_p()
        _check(lib.rime_plan_create(ctypes.byref(d), ctypes.byref(h)), "rime_plan_create")
        self.handle = h
        self._lib = lib

    def close(self):
        if getattr(self, "handle", None):
            self._lib.rime_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, mode: int, prec: int, nset: int = 1, total_src: int = 1) -> int:
        return int(self._lib.rime_workspace_size(self.handle, mode, prec, nset, total_src))

    def set_variant(self, mode: int, prec: int, index: int):
        _check(self._lib.rime_set_variant(self.handle, mode, prec, index), "rime_set_variant")

    def get_variant(self, mode: int, prec: int) -> int:
        return int(self._lib.rime_get_variant(self.handle, mode, prec))

    def set_timing_events(self, start=None, stop=None):
        """torch.cuda.Event pair recorded around the main kernel of later calls.
        torch creates an event's hipEvent on its first record(), so each event
        must have been recorded once before it is passed here."""
        for ev in (start, stop):
            if ev is not None and not ev.cuda_event:
                raise ValueError("timing event has no hipEvent yet: record() it once first")
        s = ctypes.c_void_p(start.cuda_event) if start is not None else None
        e = ctypes.c_void_p(stop.cuda_event) if stop is not None else None
        _check(self._lib.rime_plan_set_timing_events(self.handle, s, e),
               "rime_plan_set_timing_events")

    def set_main_events(self, start=None, stop=None):
        """torch.cuda.Event pair recorded around the per-baseline kernel alone
        (same creation rule as set_timing_events)."""
        for ev in (start, stop):
            if ev is not None and not ev.cuda_event:
                raise ValueError("timing event has no hipEvent yet: record() it once first")
        s = ctypes.c_void_p(start.cuda_event) if start is not None else None
        e = ctypes.c_void_p(stop.cuda_event) if stop is not None else None
        _check(self._lib.rime_plan_set_main_events(self.handle, s, e), "rime_plan_set_main_events")


@dataclass
class DeviceSky:
    """One sky model on the device: float64 CUDA tensors, points first, then
    Gaussians (gshape), then exponential disks (xshape)."""
    lm: object
    stokes: object
    alpha: object
    gshape: object
    npsrc: int
    ngsrc: int
    xshape: object = None
    nxsrc: int = 0

    @property
    def nsrc(self) -> int:
        return self.npsrc + self.ngsrc + self.nxsrc

    @staticmethod
    def from_host(sky, device="cuda"):
        import torch
        t = lambda a, shape: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(shape),
                                             device=device)
        xs = getattr(sky, "xshape", None)
        xs = np.zeros((0, 3)) if xs is None else xs
        n, ng, nx = int(sky.lm.shape[0]), int(sky.gshape.shape[0]), int(xs.shape[0])
        return DeviceSky(lm=t(sky.lm, (n, 2)), stokes=t(sky.stokes, (n, 4)),
                         alpha=t(sky.alpha, (n,)), gshape=t(sky.gshape, (ng, 3)),
                         npsrc=n - ng - nx, ngsrc=ng, xshape=t(xs, (nx, 3)), nxsrc=nx)

    def desc(self) -> SkyDesc:
        for x in (self.lm, self.stokes, self.alpha, self.gshape):
            _expect(x, "float64")
        if self.nxsrc:
            _expect(self.xshape, "float64", (self.nxsrc, 3))
        d = SkyDesc()
        d.npsrc, d.ngsrc, d.nxsrc = self.npsrc, self.ngsrc, self.nxsrc
        d.lm, d.stokes, d.alpha = (self.lm.data_ptr(), self.stokes.data_ptr(),
                                   self.alpha.data_ptr())
        d.gshape = self.gshape.data_ptr() if self.ngsrc > 0 else None
        d.xshape = self.xshape.data_ptr() if self.nxsrc > 0 else None
        return d


def _expect(x, dtype: str, shape=None):
    if not x.is_cuda:
        raise ValueError("expected a CUDA tensor")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if str(x.dtype).replace("torch.", "") != dtype:
        raise ValueError(f"expected dtype {dtype}, got {x.dtype}")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(x.shape)}")


def _vis_dtypes(prec: int):
    return ("complex128", "float64") if prec == FP64 else ("complex64", "float32")


def workspace(plan: Plan, mode: int, prec: int, nset: int = 1, total_src: int = 1, device="cuda"):
    import torch
    n = max(plan.workspace_size(mode, prec, nset, total_src), 256)
    return torch.empty(n, dtype=torch.uint8, device=device)


def rime_workspace_size(plan: Plan, mode: int, prec: int, nset: int = 1, total_src: int = 1) -> int:
    return plan.workspace_size(mode, prec, nset, total_src)


def rime_predict(plan: Plan, sky: DeviceSky, prec: int, vis, ws, stream=None):
    cdt, _ = _vis_dtypes(prec)
    _expect(vis, cdt, (plan.ntime, plan.nbl, plan.nchan, 4))
    d = sky.desc()
    _check(plan._lib.rime_predict(plan.handle, ctypes.byref(d), prec, _dptr(vis), _dptr(ws),
                                  ws.numel(), _stream(stream)), "rime_predict")


def rime_chi2(plan: Plan, sky: DeviceSky, prec: int, data, weight, chi2, ws, stream=None):
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    _expect(data, cdt, shp)
    _expect(weight, rdt, shp)
    _expect(chi2, "float64", (1,))
    d = sky.desc()
    _check(plan._lib.rime_chi2(plan.handle, ctypes.byref(d), prec, _dptr(data), _dptr(weight),
                               _dptr(chi2), _dptr(ws), ws.numel(), _stream(stream)), "rime_chi2")


def rime_chi2_grad(plan: Plan, sky: DeviceSky, prec: int, data, weight, chi2, grad, ws,
                   stream=None):
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    _expect(data, cdt, shp)
    _expect(weight, rdt, shp)
    _expect(chi2, "float64", (1,))
    _expect(grad, "float64", (sky.nsrc, 10))
    d = sky.desc()
    _check(plan._lib.rime_chi2_grad(plan.handle, ctypes.byref(d), prec, _dptr(data),
                                    _dptr(weight), _dptr(chi2), _dptr(grad), _dptr(ws),
                                    ws.numel(), _stream(stream)), "rime_chi2_grad")


def rime_chi2_grad_noalloc(plan: Plan, sky: DeviceSky, prec: int, data, weight, chi2, grad,
                           stream=None):
    """rime_chi2_grad with the library's fixed per-device workspace (no
    allocation; calls on one device must not overlap)."""
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    _expect(data, cdt, shp)
    _expect(weight, rdt, shp)
    _expect(chi2, "float64", (1,))
    _expect(grad, "float64", (sky.nsrc, 10))
    d = sky.desc()
    _check(plan._lib.rime_chi2_grad_noalloc(plan.handle, ctypes.byref(d), prec, _dptr(data),
                                            _dptr(weight), _dptr(chi2), _dptr(grad),
                                            _stream(stream)), "rime_chi2_grad_noalloc")


def rime_streamed_workspace_size(plan: Plan, mode: int, prec: int, nsrc: int,
                                 chunk_t: int) -> int:
    return int(plan._lib.rime_streamed_workspace_size(plan.handle, mode, prec, nsrc, chunk_t))


def rime_chi2_streamed(plan: Plan, sky: DeviceSky, prec: int, data_host, weight_host, chi2,
                       grad, chunk_t: int, ws, stream=None):
    """chi^2 (grad None) or chi^2 and gradient with the data and weights in
    host memory (CPU torch tensors, preferably pinned), uploaded in chunks of
    chunk_t timesteps.  The host tensors must stay alive and unchanged until
    the stream has finished the call."""
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    for x, dt in ((data_host, cdt), (weight_host, rdt)):
        if x.is_cuda or not x.is_contiguous():
            raise ValueError("expected a contiguous host tensor")
        if str(x.dtype).replace("torch.", "") != dt or tuple(x.shape) != shp:
            raise ValueError(f"expected a host {dt} tensor of shape {shp}")
    _expect(chi2, "float64", (1,))
    if grad is not None:
        _expect(grad, "float64", (sky.nsrc, 10))
    d = sky.desc()
    _check(plan._lib.rime_chi2_streamed(plan.handle, ctypes.byref(d), prec,
                                        ctypes.c_void_p(data_host.data_ptr()),
                                        ctypes.c_void_p(weight_host.data_ptr()), _dptr(chi2),
                                        _dptr(grad), int(chunk_t), _dptr(ws), ws.numel(),
                                        _stream(stream)), "rime_chi2_streamed")


def _terms(plan, sky, die=None, grad_die=None, stokes_t=None, grad_stokes_t=None):
    """TermsDesc of the optional per-call terms (device tensors): die and
    grad_die complex128 [ntime][na][nchan][2][2], stokes_t and grad_stokes_t
    float64 [ntime][nsrc][4]."""
    t = TermsDesc()
    gshape = (plan.ntime, plan.na, plan.nchan, 2, 2)
    sshape = (plan.ntime, sky.nsrc, 4)
    for name, x, dt, shp in (("die", die, "complex128", gshape),
                             ("grad_die", grad_die, "complex128", gshape),
                             ("stokes_t", stokes_t, "float64", sshape),
                             ("grad_stokes_t", grad_stokes_t, "float64", sshape)):
        if x is not None:
            _expect(x, dt, shp)
            setattr(t, name, x.data_ptr())
    return t


def rime_workspace_size_ex(plan: Plan, mode: int, prec: int, nsrc: int, die=False,
                           grad_die=False, stokes_t=False, grad_stokes_t=False) -> int:
    """Workspace bytes of a single-sky call with the given terms present."""
    t = TermsDesc()
    # presence is what counts: any non-null address
    t.die = 1 if (die or grad_die) else None
    t.grad_die = 1 if grad_die else None
    t.stokes_t = 1 if (stokes_t or grad_stokes_t) else None
    t.grad_stokes_t = 1 if grad_stokes_t else None
    return int(plan._lib.rime_workspace_size_ex(plan.handle, mode, prec, nsrc, ctypes.byref(t)))


def rime_predict_ex(plan: Plan, sky: DeviceSky, prec: int, vis, ws, die=None, stokes_t=None,
                    stream=None):
    cdt, _ = _vis_dtypes(prec)
    _expect(vis, cdt, (plan.ntime, plan.nbl, plan.nchan, 4))
    d = sky.desc()
    t = _terms(plan, sky, die=die, stokes_t=stokes_t)
    _check(plan._lib.rime_predict_ex(plan.handle, ctypes.byref(d), ctypes.byref(t), prec,
                                     _dptr(vis), _dptr(ws), ws.numel(), _stream(stream)),
           "rime_predict_ex")


def rime_chi2_ex(plan: Plan, sky: DeviceSky, prec: int, data, weight, chi2, grad, ws, die=None,
                 grad_die=None, stokes_t=None, grad_stokes_t=None, stream=None):
    """chi^2 (grad None) or chi^2 and gradient with the per-call terms."""
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    _expect(data, cdt, shp)
    _expect(weight, rdt, shp)
    _expect(chi2, "float64", (1,))
    if grad is not None:
        _expect(grad, "float64", (sky.nsrc, 10))
    d = sky.desc()
    t = _terms(plan, sky, die, grad_die, stokes_t, grad_stokes_t)
    _check(plan._lib.rime_chi2_ex(plan.handle, ctypes.byref(d), ctypes.byref(t), prec,
                                  _dptr(data), _dptr(weight), _dptr(chi2), _dptr(grad),
                                  _dptr(ws), ws.numel(), _stream(stream)), "rime_chi2_ex")


class Batch:
    """rime_batch_create over a list of DeviceSky (their tensors must stay
    alive and keep their addresses; overwrite values in place)."""

    def __init__(self, plan: Plan, skies):
        self.plan = plan
        self.skies = list(skies)
        arr = (SkyDesc * len(self.skies))(*[s.desc() for s in self.skies])
        h = ctypes.c_void_p()
        _check(plan._lib.rime_batch_create(plan.handle, len(self.skies), arr, ctypes.byref(h)),
               "rime_batch_create")
        self.handle = h
        self.total_src = sum(s.nsrc for s in self.skies)

    def workspace_size(self, mode: int, prec: int) -> int:
        return int(self.plan._lib.rime_batch_workspace_size(self.handle, mode, prec))

    def close(self):
        if getattr(self, "handle", None):
            self.plan._lib.rime_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rime_batch_create(plan: Plan, skies) -> Batch:
    return Batch(plan, skies)


def rime_chi2_batched(batch: Batch, prec: int, data, weight, chi2, grad, ws, stream=None,
                      use_graph: bool = False):
    plan = batch.plan
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    _expect(data, cdt, shp)
    _expect(weight, rdt, shp)
    _expect(chi2, "float64", (len(batch.skies),))
    if grad is not None:
        _expect(grad, "float64", (batch.total_src, 10))
    _check(plan._lib.rime_chi2_batched(batch.handle, prec, _dptr(data), _dptr(weight),
                                       _dptr(chi2), _dptr(grad), _dptr(ws), ws.numel(),
                                       _stream(stream), 1 if use_graph else 0),
           "rime_chi2_batched")


def rime_variant_matrix_cores(mode: int, prec: int, index: int) -> bool:
    """Whether the variant forms the point-source sums on the matrix cores."""
    r = int(load_library().rime_variant_matrix_cores(mode, prec, index))
    if r < 0:
        raise RimeError(1, f"rime_variant_matrix_cores: no variant {index} for mode {mode}, "
                           f"precision {prec}")
    return bool(r)


def rime_domain_status(ws, stream=None) -> int:
    """Status of the domain check of the last call that used workspace `ws`
    (synchronises `stream` first): 0 when every source had l^2 + m^2 < 1,
    RIME_ERR_DOMAIN (6) when one did; raises RimeError on any other status."""
    st = int(load_library().rime_domain_status(_dptr(ws), ws.numel(), _stream(stream)))
    if st not in (0, RIME_ERR_DOMAIN):
        raise RimeError(st, "rime_domain_status")
    return st


def rime_batch_autotune(batch: Batch, mode: int, prec: int, data, weight, ws):
    plan = batch.plan
    cdt, rdt = _vis_dtypes(prec)
    shp = (plan.ntime, plan.nbl, plan.nchan, 4)
    _expect(data, cdt, shp)
    _expect(weight, rdt, shp)
    _check(plan._lib.rime_batch_autotune(batch.handle, mode, prec, _dptr(data), _dptr(weight),
                                         _dptr(ws), ws.numel()), "rime_batch_autotune")


def rime_batch_set_variant(batch: Batch, mode: int, prec: int, index: int):
    _check(batch.plan._lib.rime_batch_set_variant(batch.handle, mode, prec, index),
           "rime_batch_set_variant")


def rime_batch_get_variant(batch: Batch, mode: int, prec: int) -> int:
    return int(batch.plan._lib.rime_batch_get_variant(batch.handle, mode, prec))


def rime_autotune(plan: Plan, sky: DeviceSky, mode: int, prec: int, data, weight, ws,
                  cache_path: str | None = None):
    """Time every compiled variant on this sky and keep the fastest; the choice
    is cached in `cache_path` (default: the file named by RIME_TUNE_CACHE, if
    set)."""
    d = sky.desc()
    cache_path = cache_path or os.environ.get("RIME_TUNE_CACHE")
    cp = cache_path.encode() if cache_path else None
    _check(plan._lib.rime_autotune(plan.handle, ctypes.byref(d), mode, prec,
                                   _dptr(data) if data is not None else None,
                                   _dptr(weight) if weight is not None else None,
                                   _dptr(ws), ws.numel(), cp), "rime_autotune")


def rime_loglike_const(weight: np.ndarray) -> float:
    lib = load_library()
    w = np.ascontiguousarray(weight, dtype=np.float64).reshape(-1)
    return float(lib.rime_loglike_const(_f64p(w), w.size))


def rime_variant_count(mode: int, prec: int) -> int:
    return int(load_library().rime_variant_count(mode, prec))


def rime_variant_info(mode: int, prec: int, index: int):
    lib = load_library()
    t, c, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.rime_variant_info(mode, prec, index, ctypes.byref(t), ctypes.byref(c),
                                 ctypes.byref(s)), "rime_variant_info")
    return t.value, c.value, s.value


def rime_tiling_host(na: int, ant1, ant2, threads: int):
    """Host-only tiling (no GPU needed): returns (tile_bl, tile_lpq, tile_ant)."""
    lib = load_library()
    a1 = np.ascontiguousarray(ant1, dtype=np.int32)
    a2 = np.ascontiguousarray(ant2, dtype=np.int32)
    nt = ctypes.c_int32()
    _check(lib.rime_tiling_host(na, a1.size, _i32p(a1), _i32p(a2), threads, 0, ctypes.byref(nt),
                                None, None, None), "rime_tiling_host")
    nat = 64 if threads >= 1024 else 32 if threads >= 256 else 16
    bl = np.empty((nt.value, threads), np.int32)
    lpq = np.empty((nt.value, threads), np.int32)
    ant = np.empty((nt.value, nat), np.int32)
    _check(lib.rime_tiling_host(na, a1.size, _i32p(a1), _i32p(a2), threads, nt.value,
                                ctypes.byref(nt), _i32p(bl), _i32p(lpq), _i32p(ant)),
           "rime_tiling_host")
    return bl, lpq, ant
