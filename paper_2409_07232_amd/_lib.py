"""ctypes binding of the C ABI in ``include/fsbm_coal.h``.

Argument marshalling only: every step of the collision path runs in the HIP
library ``libfsbm_coal.so``.  Device memory and streams come from PyTorch
(``torch.Tensor.data_ptr()``, ``torch.cuda.Stream.cuda_stream``).  There is no
CPU fallback: if the library is missing, loading fails loudly.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsbm_coal.so")

FSBM_OK = 0
FSBM_EINVAL = -1
FSBM_ENOMEM = -2
FSBM_EHIP = -3
FSBM_EUNSUPPORTED = -4
FSBM_EDOMAIN = -5
FSBM_FP64 = 0
FSBM_FP32C = 1
ORDER_SIMULTANEOUS = 0
ORDER_SEQUENTIAL = 1
FLAG_DEBUG_CHECKS = 1
FLAG_NO_GRAPH = 2
FLAG_FORCE_WAVE = 4
FLAG_PROFILE = 8

# every entry point declared in include/fsbm_coal.h
EXPORTS = ("fsbm_coal_opts_default", "fsbm_coal_create", "fsbm_coal_step",
           "fsbm_coal_step_gated", "fsbm_coal_step_noalloc",
           "fsbm_coal_sediment", "fsbm_coal_condense",
           "fsbm_coal_set_breakup", "fsbm_coal_breakup",
           "fsbm_coal_step_multi", "fsbm_coal_tune", "fsbm_coal_totals",
           "fsbm_coal_get_stats", "fsbm_coal_destroy", "fsbm_coal_strerror",
           "fsbm_coal_last_error")


class FsbmError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        msg = "%s failed: %s (%d)" % (where, strerror(code), code)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


class Opts(ctypes.Structure):
    _fields_ = [("x1_g", ctypes.c_double),
                ("s", ctypes.c_int32),
                ("product", ctypes.POINTER(ctypes.c_int32)),
                ("precision", ctypes.c_int32),
                ("theta", ctypes.c_double),
                ("steps_per_launch", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("order", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("active_points", ctypes.c_int64),
                ("pair_evals", ctypes.c_int64),
                ("limiter_steps", ctypes.c_int64),
                ("fp64_fallback_steps", ctypes.c_int64),
                ("kernel", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32),
                ("kernel_launches", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double),
                ("exact_pair_evals", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64),
                ("tune_candidates", ctypes.c_int32),
                ("tune_rejected", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            "libfsbm_coal.so is missing; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.fsbm_coal_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.fsbm_coal_opts_default.restype = None
    lib.fsbm_coal_create.argtypes = [ctypes.c_int32, ctypes.c_int32, dp,
                                     ctypes.c_int32, dp,
                                     ctypes.POINTER(Opts),
                                     ctypes.POINTER(vp)]
    lib.fsbm_coal_create.restype = ctypes.c_int
    lib.fsbm_coal_step.argtypes = [vp, vp, vp, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_int32, vp]
    lib.fsbm_coal_step.restype = ctypes.c_int
    lib.fsbm_coal_step_gated.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64,
                                         ctypes.c_double, ctypes.c_int32, vp]
    lib.fsbm_coal_step_gated.restype = ctypes.c_int
    lib.fsbm_coal_step_noalloc.argtypes = [vp, vp, vp, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_int32,
                                           vp]
    lib.fsbm_coal_step_noalloc.restype = ctypes.c_int
    lib.fsbm_coal_step_multi.argtypes = [ctypes.POINTER(vp), ctypes.c_int32,
                                         ctypes.POINTER(vp),
                                         ctypes.POINTER(vp),
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_double, ctypes.c_int32, vp]
    lib.fsbm_coal_step_multi.restype = ctypes.c_int
    lib.fsbm_coal_sediment.argtypes = [vp, vp, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int64, vp, vp, vp,
                                       ctypes.c_double, ctypes.c_int32, vp,
                                       vp]
    lib.fsbm_coal_sediment.restype = ctypes.c_int
    lib.fsbm_coal_condense.argtypes = [vp, vp, ctypes.c_int64, vp, vp,
                                       ctypes.c_double, ctypes.c_int32, vp,
                                       vp]
    lib.fsbm_coal_condense.restype = ctypes.c_int
    lib.fsbm_coal_set_breakup.argtypes = [vp, dp, dp]
    lib.fsbm_coal_set_breakup.restype = ctypes.c_int
    lib.fsbm_coal_breakup.argtypes = [vp, vp, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_int32, vp]
    lib.fsbm_coal_breakup.restype = ctypes.c_int
    lib.fsbm_coal_tune.argtypes = [vp, ctypes.c_int64, vp]
    lib.fsbm_coal_tune.restype = ctypes.c_int
    lib.fsbm_coal_totals.argtypes = [vp, vp, vp, vp, vp]
    lib.fsbm_coal_totals.restype = ctypes.c_int
    lib.fsbm_coal_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.fsbm_coal_get_stats.restype = ctypes.c_int
    lib.fsbm_coal_destroy.argtypes = [vp]
    lib.fsbm_coal_destroy.restype = ctypes.c_int
    lib.fsbm_coal_strerror.argtypes = [ctypes.c_int]
    lib.fsbm_coal_strerror.restype = ctypes.c_char_p
    lib.fsbm_coal_last_error.argtypes = [vp]
    lib.fsbm_coal_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().fsbm_coal_strerror(int(code)).decode()


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check_state(N, S, B):
    import torch
    if not isinstance(N, torch.Tensor) or N.dtype != torch.float64:
        raise TypeError("N must be a float64 torch tensor")
    if not N.is_cuda or not N.is_contiguous():
        raise ValueError("N must be a contiguous device tensor")
    if N.dim() != 3 or N.shape[1] != S or N.shape[2] != B:
        raise ValueError("N must have shape [npoints, %d, %d]" % (S, B))


def _check_p(p, P):
    import torch
    if not isinstance(p, torch.Tensor) or p.dtype != torch.float64:
        raise TypeError("p must be a float64 torch tensor")
    if not p.is_cuda or not p.is_contiguous() or p.shape != (P,):
        raise ValueError("p must be a contiguous device tensor of [npoints]")


class FsbmCoal:
    """One bin grid and species set (``fsbm_coal_create``)."""

    def __init__(self, nbins: int, nspecies: int, kernel_tables,
                 p_levels, *, x1_g: Optional[float] = None, s: int = 1,
                 product=None, precision: int = FSBM_FP64,
                 theta: float = 1e-30, steps_per_launch: int = 0,
                 flags: int = 0, order: int = ORDER_SIMULTANEOUS):
        lib = load()
        self.nbins, self.nspecies = int(nbins), int(nspecies)
        self.precision = int(precision)
        tables = np.ascontiguousarray(kernel_tables, dtype=np.float64)
        plev = np.ascontiguousarray(p_levels, dtype=np.float64)
        opts = Opts()
        lib.fsbm_coal_opts_default(ctypes.byref(opts))
        if x1_g is not None:
            opts.x1_g = float(x1_g)
        opts.s = int(s)
        opts.precision = self.precision
        opts.theta = float(theta)
        opts.steps_per_launch = int(steps_per_launch)
        opts.order = int(order)
        opts.flags = int(flags)
        prod = None
        if product is not None:
            prod = np.ascontiguousarray(product, dtype=np.int32)
            opts.product = prod.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        h = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        rc = lib.fsbm_coal_create(self.nbins, self.nspecies,
                                  tables.ctypes.data_as(dp),
                                  int(plev.shape[0]), plev.ctypes.data_as(dp),
                                  ctypes.byref(opts), ctypes.byref(h))
        if rc != FSBM_OK:
            raise FsbmError(rc, "fsbm_coal_create")
        self._h = h
        self._last_npoints = 0

    @classmethod
    def from_workload(cls, w, precision=FSBM_FP64, **kw):
        return cls(w.nbins, w.nspecies, w.tables, w.p_levels, x1_g=w.x1_g,
                   s=w.s, product=w.product if w.nspecies > 1 else None,
                   precision=precision, theta=w.theta, **kw)

    @property
    def handle(self):
        return self._h

    def _raise(self, rc, where):
        detail = load().fsbm_coal_last_error(self._h).decode()
        raise FsbmError(rc, where, detail)

    def step(self, N, p, dt: float, nsteps: int, stream=None):
        """Advance N ([P][S][B] float64, device) in place."""
        _check_state(N, self.nspecies, self.nbins)
        P = int(N.shape[0])
        _check_p(p, P)
        rc = load().fsbm_coal_step(self._h, N.data_ptr(), p.data_ptr(), P,
                                   float(dt), int(nsteps),
                                   _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_step")
        self._last_npoints = P

    def step_gated(self, N, p, t_old, t_now, dt: float, nsteps: int,
                   stream=None):
        """step() with the temperature gates (``fsbm_coal_step_gated``):
        t_old / t_now are [P] float64 device tensors (K) or None."""
        _check_state(N, self.nspecies, self.nbins)
        P = int(N.shape[0])
        _check_p(p, P)
        ptrs = []
        for t in (t_old, t_now):
            if t is None:
                ptrs.append(None)
            else:
                _check_p(t, P)
                ptrs.append(t.data_ptr())
        rc = load().fsbm_coal_step_gated(self._h, N.data_ptr(), p.data_ptr(),
                                         ptrs[0], ptrs[1], P, float(dt),
                                         int(nsteps), _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_step_gated")
        self._last_npoints = P

    def step_noalloc(self, N, p, dt: float, nsteps: int, stream=None):
        """Same as step() through ``fsbm_coal_step_noalloc``: the library's
        static scratch block is the workspace, nothing is allocated."""
        _check_state(N, self.nspecies, self.nbins)
        P = int(N.shape[0])
        _check_p(p, P)
        rc = load().fsbm_coal_step_noalloc(self._h, N.data_ptr(),
                                           p.data_ptr(), P, float(dt),
                                           int(nsteps),
                                           _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_step_noalloc")
        self._last_npoints = P

    def sediment(self, N, ncols: int, nlev: int, col_stride: int,
                 lev_stride: int, dz_cm, v_cm_s, vfac, dt: float,
                 nsteps: int, precip=None, stream=None):
        """Sedimentation of columns of N (``fsbm_coal_sediment``): dz_cm
        [nlev], v_cm_s [S][B], vfac [ncols][nlev] or None, precip
        [ncols][S][B] or None, all float64 device tensors."""
        _check_state(N, self.nspecies, self.nbins)
        P = int(N.shape[0])
        if ncols > 0 and ((ncols - 1) * col_stride + (nlev - 1) * lev_stride
                          >= P):
            raise ValueError("columns reach past the state array")
        shapes = ((dz_cm, (nlev,)), (v_cm_s, (self.nspecies, self.nbins)),
                  (vfac, (ncols, nlev)),
                  (precip, (ncols, self.nspecies, self.nbins)))
        for t, shp in shapes:
            if t is not None and (t.dtype != N.dtype or not t.is_cuda or
                                  not t.is_contiguous() or
                                  tuple(t.shape) != shp):
                raise ValueError("sediment: array of shape %s expected" %
                                 (shp,))
        ptr = [None if t is None else t.data_ptr()
               for t in (dz_cm, v_cm_s, vfac, precip)]
        rc = load().fsbm_coal_sediment(self._h, N.data_ptr(), int(ncols),
                                       int(nlev), int(col_stride),
                                       int(lev_stride), ptr[0], ptr[1],
                                       ptr[2], float(dt), int(nsteps), ptr[3],
                                       _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_sediment")

    def condense(self, N, ssat, gcoef_cm2_s, dt: float, nsteps: int,
                 evaporated=None, stream=None):
        """Condensation/evaporation of species 0 (``fsbm_coal_condense``):
        ssat and gcoef_cm2_s [npoints], evaporated [npoints] or None, all
        float64 device tensors."""
        _check_state(N, self.nspecies, self.nbins)
        P = int(N.shape[0])
        for t in (ssat, gcoef_cm2_s, evaporated):
            if t is not None and (t.dtype != N.dtype or not t.is_cuda or
                                  not t.is_contiguous() or
                                  tuple(t.shape) != (P,)):
                raise ValueError("condense: array of shape (%d,) expected" % P)
        rc = load().fsbm_coal_condense(
            self._h, N.data_ptr(), P, ssat.data_ptr(),
            gcoef_cm2_s.data_ptr(), float(dt), int(nsteps),
            None if evaporated is None else evaporated.data_ptr(),
            _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_condense")

    def set_breakup(self, rate_per_s, fragments):
        """Breakup rates [B] and fragment table [B][B] (host arrays,
        ``fsbm_coal_set_breakup``)."""
        import numpy as np
        B = self.nbins
        r = np.ascontiguousarray(rate_per_s, dtype=np.float64)
        q = np.ascontiguousarray(fragments, dtype=np.float64)
        if r.shape != (B,) or q.shape != (B, B):
            raise ValueError("rates [%d] and fragments [%d][%d] expected" %
                             (B, B, B))
        dp = ctypes.POINTER(ctypes.c_double)
        rc = load().fsbm_coal_set_breakup(self._h, r.ctypes.data_as(dp),
                                          q.ctypes.data_as(dp))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_set_breakup")

    def breakup(self, N, dt: float, nsteps: int, stream=None):
        """Spontaneous breakup of species 0 (``fsbm_coal_breakup``)."""
        _check_state(N, self.nspecies, self.nbins)
        rc = load().fsbm_coal_breakup(self._h, N.data_ptr(), int(N.shape[0]),
                                      float(dt), int(nsteps),
                                      _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_breakup")

    def totals(self):
        """Per-point (mass_before, mass_after, num_before, num_after)."""
        import torch
        P = self._last_npoints
        out = [torch.empty(P, dtype=torch.float64, device="cuda")
               for _ in range(4)]
        rc = load().fsbm_coal_totals(self._h, *[o.data_ptr() for o in out])
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_totals")
        return tuple(out)

    def stats(self) -> dict:
        st = Stats()
        rc = load().fsbm_coal_get_stats(self._h, ctypes.byref(st))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_get_stats")
        return {f: getattr(st, f) for f, _ in Stats._fields_}

    def tune(self, npoints_hint: int, stream=None):
        rc = load().fsbm_coal_tune(self._h, int(npoints_hint),
                                   _stream_handle(stream))
        if rc != FSBM_OK:
            self._raise(rc, "fsbm_coal_tune")

    def close(self):
        if getattr(self, "_h", None):
            load().fsbm_coal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_multi(handles: Sequence[FsbmCoal], Ns, ps, dt: float, nsteps: int,
               stream=None):
    """One launch sequence over several grids (``fsbm_coal_step_multi``)."""
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.handle for h in handles])
    nptr = (ctypes.c_void_p * n)()
    pptr = (ctypes.c_void_p * n)()
    cnt = (ctypes.c_int64 * n)()
    for g, (h, N, p) in enumerate(zip(handles, Ns, ps)):
        _check_state(N, h.nspecies, h.nbins)
        _check_p(p, int(N.shape[0]))
        nptr[g] = N.data_ptr()
        pptr[g] = p.data_ptr()
        cnt[g] = int(N.shape[0])
        h._last_npoints = int(N.shape[0])
    rc = load().fsbm_coal_step_multi(hs, n, nptr, pptr, cnt, float(dt),
                                     int(nsteps), _stream_handle(stream))
    if rc != FSBM_OK:
        raise FsbmError(rc, "fsbm_coal_step_multi")
