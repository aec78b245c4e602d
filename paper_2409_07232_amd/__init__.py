"""MI355X (gfx950) collision-coalescence step of the FSBM bin microphysics.

The HIP library (``libfsbm_coal.so``, sources in ``csrc/``) is loaded lazily
by :mod:`paper_2409_07232_amd._lib`; importing this package does not touch
the GPU.  ``workloads`` builds seeded synthetic inputs.
"""

__all__ = ["FsbmCoal", "step_multi", "FSBM_FP64", "FSBM_FP32C", "load"]


def __getattr__(name):
    if name in ("FsbmCoal", "step_multi", "FSBM_FP64", "FSBM_FP32C", "load",
                "FsbmError", "FLAG_NO_GRAPH", "FLAG_DEBUG_CHECKS",
                "FLAG_FORCE_WAVE"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
