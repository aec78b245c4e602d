"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every entry point declared in include/fsbm_coal.h, and the pure-host
entry points behave as documented."""

import ctypes
import os
import re

import pytest

from paper_2409_07232_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fsbm_coal.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsbm_coal_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_strerror_and_defaults():
    assert _lib.strerror(0) == "success"
    assert "invalid" in _lib.strerror(_lib.FSBM_EINVAL)
    assert "unsupported" in _lib.strerror(_lib.FSBM_EUNSUPPORTED)
    assert _lib.strerror(-99) == "unknown error"
    o = _lib.Opts()
    _lib.load().fsbm_coal_opts_default(ctypes.byref(o))
    assert o.s == 1 and o.precision == _lib.FSBM_FP64
    assert o.theta == 1e-30
    assert abs(o.x1_g - 3.3510321638291124e-11) < 1e-25


def test_null_arguments_rejected_without_device_work():
    lib = _lib.load()
    assert lib.fsbm_coal_create(33, 1, None, 1, None, None, None) == \
        _lib.FSBM_EINVAL
    assert lib.fsbm_coal_step(None, None, None, 10, 1.0, 1, None) == \
        _lib.FSBM_EINVAL
    assert lib.fsbm_coal_destroy(None) == 0
    assert lib.fsbm_coal_last_error(None) == b""


def test_no_cpu_fallback_in_binding():
    src = open(os.path.join(ROOT, "paper_2409_07232_amd", "_lib.py")).read()
    assert "oracle" not in src
    with pytest.raises(FileNotFoundError):
        _lib.load.__wrapped__ if hasattr(_lib.load, "__wrapped__") else None
        saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load("/nonexistent/libfsbm_coal.so")
        finally:
            _lib._lib = saved


def _create(nbins, nspecies, opts):
    import numpy as np
    lib = _lib.load()
    npairs = nspecies * (nspecies + 1) // 2
    tables = np.full(npairs * nbins * nbins, 1e-4)
    plev = np.array([1000.0])
    dp = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    prod = (ctypes.c_int32 * (nspecies * nspecies))()
    if nspecies > 1:
        opts.product = ctypes.cast(prod, ctypes.POINTER(ctypes.c_int32))
    return lib.fsbm_coal_create(nbins, nspecies, tables.ctypes.data_as(dp), 1,
                                plev.ctypes.data_as(dp), ctypes.byref(opts),
                                ctypes.byref(h))


def test_sequential_order_shapes_rejected_without_device_work():
    """The sequential form exists for one species on the doubling grid in
    FP64 with the lane kernel's bin counts; everything else is refused at
    create time, before any device call."""
    lib = _lib.load()
    o = _lib.Opts()
    lib.fsbm_coal_opts_default(ctypes.byref(o))
    assert o.order == _lib.ORDER_SIMULTANEOUS
    o.order = _lib.ORDER_SEQUENTIAL
    o.precision = _lib.FSBM_FP32C
    assert _create(33, 1, o) == _lib.FSBM_EUNSUPPORTED
    o.precision = _lib.FSBM_FP64
    assert _create(33, 2, o) == _lib.FSBM_EUNSUPPORTED
    assert _create(66, 1, o) == _lib.FSBM_EUNSUPPORTED      # not a lane size
    o.s = 2
    assert _create(33, 1, o) == _lib.FSBM_EUNSUPPORTED      # refined grid
    o.s = 1
    o.flags = _lib.FLAG_FORCE_WAVE
    assert _create(33, 1, o) == _lib.FSBM_EUNSUPPORTED
    o.flags = 0
    o.order = 7
    assert _create(33, 1, o) == _lib.FSBM_EINVAL


def test_shapes_beyond_the_kernels_rejected_without_device_work():
    """S x B above 64 lanes x 12 bins (the one-point-per-wave kernel's
    largest shape), more than 512 bins or more than 8 species are refused
    at create time, before any device call."""
    lib = _lib.load()
    o = _lib.Opts()
    lib.fsbm_coal_opts_default(ctypes.byref(o))
    o.s = 12
    assert _create(400, 2, o) == _lib.FSBM_EUNSUPPORTED
    o.s = 1
    assert _create(97, 8, o) == _lib.FSBM_EUNSUPPORTED
    assert _create(513, 1, o) == _lib.FSBM_EUNSUPPORTED
    assert _create(33, 9, o) == _lib.FSBM_EINVAL


def _create_with(nbins=8, nspecies=1, tables=None, levels=(1000.0,),
                 product=None, **opt):
    """fsbm_coal_create with every argument settable; returns its code.  Only
    invalid combinations are passed, which are refused before any device
    call."""
    import numpy as np
    lib = _lib.load()
    npairs = nspecies * (nspecies + 1) // 2
    L = len(levels)
    if tables is None:
        tables = np.full(npairs * L * nbins * nbins, 1e-4)
    tables = np.ascontiguousarray(tables, dtype=np.float64)
    plev = np.ascontiguousarray(levels, dtype=np.float64)
    o = _lib.Opts()
    lib.fsbm_coal_opts_default(ctypes.byref(o))
    for k, v in opt.items():
        setattr(o, k, v)
    keep = None
    if product is not None:
        keep = (ctypes.c_int32 * len(product))(*product)
        o.product = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
    dp = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    return lib.fsbm_coal_create(nbins, nspecies, tables.ctypes.data_as(dp), L,
                                plev.ctypes.data_as(dp), ctypes.byref(o),
                                ctypes.byref(h))


def test_invalid_create_arguments_rejected_without_device_work():
    """Every argument fsbm_coal_create documents as FSBM_EINVAL, one at a
    time: sizes, pressure levels (order, finiteness), table entries
    (negative, NaN, infinite), product map (range, symmetry, missing for
    S > 1), grid and option values."""
    import numpy as np
    E = _lib.FSBM_EINVAL
    assert _create_with(nbins=1) == E
    assert _create_with(nspecies=0) == E
    assert _create_with(levels=()) == E
    assert _create_with(levels=(750.0, 1000.0)) == E       # not decreasing
    assert _create_with(levels=(1000.0, 1000.0)) == E      # not strictly
    assert _create_with(levels=(1000.0, np.nan)) == E
    for v in (-1e-9, np.nan, np.inf):
        t = np.full(8 * 8, 1e-4)
        t[17] = v
        assert _create_with(tables=t) == E, v
    assert _create_with(nspecies=2) == E                   # no product map
    assert _create_with(nspecies=2, product=[0, 1, 0, 1]) == E  # asymmetric
    assert _create_with(nspecies=2, product=[0, 2, 2, 1]) == E  # out of range
    assert _create_with(nspecies=2, product=[0, -1, -1, 1]) == E
    assert _create_with(x1_g=0.0) == E
    assert _create_with(x1_g=float("inf")) == E
    assert _create_with(s=0) == E
    assert _create_with(theta=-1.0) == E
    assert _create_with(theta=float("nan")) == E
    assert _create_with(precision=7) == E
    assert _create_with(steps_per_launch=-1) == E
