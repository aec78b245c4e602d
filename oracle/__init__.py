"""FP64 CPU oracle of the FSBM collision-coalescence step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the GPU library (``paper_2409_07232_amd``) and the GPU library
never imports it.

The arithmetic lives in ``fsbm_oracle.c`` (plain loops, FP64, built with
``-ffp-contract=off``); this module only builds it with gcc and marshals
numpy arrays through ctypes.  ``closed_forms`` holds the analytic solutions
of the collection equation used to pin the oracle.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "fsbm_oracle.c"),
        os.path.join(_HERE, "fsbm_oracle_sed.c"),
        os.path.join(_HERE, "fsbm_oracle_cond.c"),
        os.path.join(_HERE, "fsbm_oracle_break.c")]

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra"]
# With FSBM_ORACLE_SANITIZE=1 the oracle is built and loaded with the
# address and undefined-behaviour checkers (a CPU build; the Python process
# must preload the address checker's runtime, see tests/test_oracle_asan.py)
SANITIZE = os.environ.get("FSBM_ORACLE_SANITIZE", "") == "1"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]
_LIB = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else
                    "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc (or the
    checked build ``liboracle_san.so``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *CFLAGS, *(SAN_FLAGS if SANITIZE else []), *_SRC,
               "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [
        ("nbins", ctypes.c_int32),
        ("nspecies", ctypes.c_int32),
        ("nlevels", ctypes.c_int32),
        ("s", ctypes.c_int32),
        ("x1_g", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("tables", ctypes.POINTER(ctypes.c_double)),
        ("p_levels", ctypes.POINTER(ctypes.c_double)),
        ("product", ctypes.POINTER(ctypes.c_int32)),
        ("order", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.fsbm_oracle_run.argtypes = [ctypes.POINTER(_Desc), dp, dp,
                                        ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_int32, dp, dp, dp, dp, lp,
                                        ip, ctypes.POINTER(ctypes.c_uint8),
                                        ctypes.c_int32]
        lib.fsbm_oracle_run.restype = ctypes.c_int
        lib.fsbm_oracle_run_gated.argtypes = [
            ctypes.POINTER(_Desc), dp, dp, dp, dp, ctypes.c_int64,
            ctypes.c_double, ctypes.c_int32, dp, dp, dp, dp, lp, ip,
            ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32]
        lib.fsbm_oracle_run_gated.restype = ctypes.c_int
        lib.fsbm_oracle_sediment.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
            ctypes.c_int64, ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double,
            ctypes.c_int32, dp]
        lib.fsbm_oracle_sediment.restype = ctypes.c_int
        lib.fsbm_oracle_condense.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
            ctypes.c_int64, dp, dp, dp, ctypes.c_double, ctypes.c_int32, dp]
        lib.fsbm_oracle_condense.restype = ctypes.c_int
        lib.fsbm_oracle_breakup.argtypes = [
            ctypes.c_int32, ctypes.c_int64, dp, dp, dp, ctypes.c_double,
            ctypes.c_int32]
        lib.fsbm_oracle_breakup.restype = ctypes.c_int
        lib.fsbm_oracle_grid.argtypes = [ctypes.POINTER(_Desc), dp]
        lib.fsbm_oracle_grid.restype = ctypes.c_int
        lib.fsbm_oracle_targets.argtypes = [ctypes.POINTER(_Desc), ip, dp]
        lib.fsbm_oracle_targets.restype = ctypes.c_int
        lib.fsbm_oracle_flux_fraction.argtypes = [ctypes.c_double,
                                                  ctypes.c_double]
        lib.fsbm_oracle_flux_fraction.restype = ctypes.c_double
        lib.fsbm_oracle_kernel_at.argtypes = [ctypes.POINTER(_Desc),
                                              ctypes.c_double, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32]
        lib.fsbm_oracle_kernel_at.restype = ctypes.c_double
        lib.fsbm_oracle_max_threads.argtypes = []
        lib.fsbm_oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class OracleModel:
    """Create-time description of one bin grid and its species set."""

    nbins: int
    nspecies: int
    tables: np.ndarray           # [S(S+1)/2][L][B][B] float64
    p_levels: np.ndarray         # [L] float64, strictly decreasing
    product: np.ndarray          # [S][S] int32
    x1_g: float = 3.3510321638291124e-11
    s: int = 1
    theta: float = 1e-30
    order: int = 0               # 0 simultaneous, 1 sequential (S == 1)

    def __post_init__(self):
        self.tables = np.ascontiguousarray(self.tables, dtype=np.float64)
        self.p_levels = np.ascontiguousarray(self.p_levels, dtype=np.float64)
        self.product = np.ascontiguousarray(self.product, dtype=np.int32)
        self.nlevels = int(self.p_levels.shape[0])
        self._desc = _Desc(
            self.nbins, self.nspecies, self.nlevels, self.s, self.x1_g,
            self.theta, _dptr(self.tables), _dptr(self.p_levels),
            self.product.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            int(self.order))

    def grid(self) -> np.ndarray:
        x = np.empty(self.nbins)
        if _load().fsbm_oracle_grid(ctypes.byref(self._desc), _dptr(x)):
            raise ValueError("bad oracle description")
        return x

    def targets(self):
        k = np.empty((self.nbins, self.nbins), dtype=np.int32)
        c = np.empty((self.nbins, self.nbins))
        rc = _load().fsbm_oracle_targets(
            ctypes.byref(self._desc),
            k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(c))
        if rc:
            raise ValueError("bad oracle description")
        return k, c

    def kernel_at(self, p, a, b, i, j) -> float:
        return _load().fsbm_oracle_kernel_at(ctypes.byref(self._desc),
                                             float(p), a, b, i, j)

    def run(self, N: np.ndarray, p: np.ndarray, dt: float, nsteps: int,
            nthreads: int = 0, totals: bool = False, t_old=None, t_now=None):
        """Advance ``N`` ([P][S][B] float64, modified in place).  With
        t_old / t_now ([P] temperatures in K), only the points with
        t_old > 193.15 and t_now > 223.15 take part."""
        if N.dtype != np.float64 or not N.flags.c_contiguous:
            raise ValueError("N must be C-contiguous float64")
        P = int(N.shape[0])
        if N.size != P * self.nspecies * self.nbins:
            raise ValueError("N has the wrong shape")
        p = np.ascontiguousarray(p, dtype=np.float64)
        if p.shape[0] != P:
            raise ValueError("p has the wrong length")
        outs = [np.empty(P) for _ in range(4)] if totals else [None] * 4
        lim = ctypes.c_int64(0)
        lim_pt = np.zeros(P, dtype=np.int32)
        lim_bins = np.zeros(N.shape, dtype=np.uint8)
        temps = []
        for t in (t_old, t_now):
            if t is not None:
                t = np.ascontiguousarray(t, dtype=np.float64)
                if t.shape != (P,):
                    raise ValueError("temperatures must be [npoints]")
            temps.append(t)
        rc = _load().fsbm_oracle_run_gated(
            ctypes.byref(self._desc), _dptr(N), _dptr(p),
            *[(_dptr(t) if t is not None else None) for t in temps], P,
            float(dt),
            int(nsteps), *[(_dptr(o) if o is not None else None)
                           for o in outs], ctypes.byref(lim),
            lim_pt.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            lim_bins.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
            int(nthreads))
        if rc:
            raise ValueError("oracle rejected its input")
        # limited_bins: [P][S][B] bool, bins the limiter scaled (sigma < 1)
        # at some step, or (sequential form) bins a cap emptied
        if self.order == 1:
            res = {"capped_pairs": int(lim.value), "capped_per_point": lim_pt}
        else:
            res = {"limiter_steps": int(lim.value),
                   "limiter_per_point": lim_pt}
        res["limited_bins"] = lim_bins.astype(bool)
        if totals:
            res.update({"mass_before": outs[0], "mass_after": outs[1],
                        "num_before": outs[2], "num_after": outs[3]})
        return res


def flux_fraction(c: float, x1: float) -> float:
    return _load().fsbm_oracle_flux_fraction(float(c), float(x1))


def max_threads() -> int:
    return int(_load().fsbm_oracle_max_threads())


def sediment(N: np.ndarray, dz_cm, v_cm_s, dt: float, nsteps: int,
             vfac=None, col_stride=None, lev_stride=None, precip=None):
    """Sedimentation of columns (``fsbm_oracle_sed.c``), ``N`` modified in
    place.  N: [points][S][B] or [columns][levels][S][B] float64; levels =
    len(dz_cm); point (column c, level l) is c * col_stride + l *
    lev_stride (default: columns of consecutive levels).  v_cm_s: [S][B];
    vfac: [columns][levels] or None.  Returns the precipitation per column,
    species and bin, added to ``precip`` if given."""
    if N.dtype != np.float64 or not N.flags.c_contiguous:
        raise ValueError("N must be C-contiguous float64")
    S, B = int(N.shape[-2]), int(N.shape[-1])
    npts = int(N.size // (S * B))
    dz = np.ascontiguousarray(dz_cm, dtype=np.float64)
    nlev = int(dz.shape[0])
    ncols = npts // nlev
    if col_stride is None:
        col_stride, lev_stride = nlev, 1
    v = np.ascontiguousarray(v_cm_s, dtype=np.float64).reshape(S, B)
    vf = None
    if vfac is not None:
        vf = np.ascontiguousarray(vfac, dtype=np.float64)
        if vf.shape != (ncols, nlev):
            raise ValueError("vfac must be [columns][levels]")
    out = (np.zeros((ncols, S, B)) if precip is None else
           np.ascontiguousarray(precip, dtype=np.float64))
    if out.shape != (ncols, S, B):
        raise ValueError("precip must be [columns][S][B]")
    rc = _load().fsbm_oracle_sediment(
        S, B, ncols, nlev, int(col_stride), int(lev_stride), _dptr(N),
        _dptr(dz), _dptr(v), _dptr(vf) if vf is not None else None,
        float(dt), int(nsteps), _dptr(out))
    if rc:
        raise ValueError("oracle rejected its input")
    return out


def condense(N: np.ndarray, ssat, gcoef_cm2_s, dt: float, nsteps: int,
             s: int = 1, x1_g: float = 3.3510321638291124e-11,
             rho: float = 1.0, evaporated=None):
    """Condensation/evaporation (``fsbm_oracle_cond.c``) of N, modified in
    place: N [points][B] (one spectrum per point) or [points][S][B] (species
    0 is the one that changes).  ssat, gcoef_cm2_s: [points].  Returns the
    evaporated mass per point (g/cm^3), added to ``evaporated`` if given."""
    if N.dtype != np.float64 or not N.flags.c_contiguous:
        raise ValueError("N must be C-contiguous float64")
    if N.ndim == 3:
        sub = np.ascontiguousarray(N[:, 0, :])
    elif N.ndim == 2:
        sub = N
    else:
        raise ValueError("N must be [points][B] or [points][S][B]")
    P, B = int(sub.shape[0]), int(sub.shape[1])
    sv = np.ascontiguousarray(ssat, dtype=np.float64)
    gv = np.ascontiguousarray(gcoef_cm2_s, dtype=np.float64)
    if sv.shape != (P,) or gv.shape != (P,):
        raise ValueError("ssat and gcoef_cm2_s must be [points]")
    out = (np.zeros(P) if evaporated is None else
           np.ascontiguousarray(evaporated, dtype=np.float64))
    if out.shape != (P,):
        raise ValueError("evaporated must be [points]")
    rc = _load().fsbm_oracle_condense(B, int(s), float(x1_g), float(rho), P,
                                      _dptr(sub), _dptr(sv), _dptr(gv),
                                      float(dt), int(nsteps), _dptr(out))
    if rc:
        raise ValueError("oracle rejected its input")
    if N.ndim == 3:
        N[:, 0, :] = sub
    return out


def breakup(N: np.ndarray, rate_per_s, fragments, dt: float, nsteps: int):
    """Spontaneous breakup (``fsbm_oracle_break.c``) of N, modified in
    place: N [points][B] or [points][S][B] (species 0 is the one that
    changes).  rate_per_s: [B]; fragments: [B][B] (row l: fragments per
    broken drop of bin l, zero on and above the diagonal)."""
    if N.dtype != np.float64 or not N.flags.c_contiguous:
        raise ValueError("N must be C-contiguous float64")
    if N.ndim == 3:
        sub = np.ascontiguousarray(N[:, 0, :])
    elif N.ndim == 2:
        sub = N
    else:
        raise ValueError("N must be [points][B] or [points][S][B]")
    P, B = int(sub.shape[0]), int(sub.shape[1])
    r = np.ascontiguousarray(rate_per_s, dtype=np.float64)
    q = np.ascontiguousarray(fragments, dtype=np.float64)
    if r.shape != (B,) or q.shape != (B, B):
        raise ValueError("rate_per_s must be [B] and fragments [B][B]")
    rc = _load().fsbm_oracle_breakup(B, P, _dptr(sub), _dptr(r), _dptr(q),
                                     float(dt), int(nsteps))
    if rc:
        raise ValueError("oracle rejected its input")
    if N.ndim == 3:
        N[:, 0, :] = sub
