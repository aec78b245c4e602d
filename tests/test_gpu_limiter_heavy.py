"""GPU parity on the first four-species recipe, where the positivity limiter
(the second pass of the step, Sec. III) fires at most points: a liquid +
crystal collision makes graupel and every species starts with the
cloud-drop spectrum, so crystals over-demand their bins within a few steps.

* 2000 points, 40 steps, FP64 and FP32C against the oracle element by
  element (the FP32C lane kernels hand each limited point to the FP64
  one-point-per-wave kernel for the rest of the call).
* 2^20 points, 100 steps as one call (the four-species size), 256 seeded
  points checked against the oracle.

Bars as in the other parity tests: rel_bin 1e-12 (FP64) / 1e-5 (FP32C),
with the oracle's limited bins on the floor the parity checker gives them,
relative mass drift 1e-10.
"""

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl
from tests.parity import check, expected_kernel, run_oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2409_07232_amd import _lib as L
    return L


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("precision", [0, 1])
def test_limiter_heavy_against_oracle(precision):
    L = _lib()
    w = wl.config3_limiter_heavy(npoints=2000, nsteps=40)
    ref, x, lim = run_oracle(w)
    assert lim.points().mean() > 0.5
    h = L.FsbmCoal.from_workload(w, precision=precision)
    N = _dev(w.N)
    h.step(N, _dev(w.p), w.dt, w.nsteps)
    torch.cuda.synchronize()
    got = N.cpu().numpy()
    st = h.stats()
    h.close()
    print("limiter-heavy precision=%d: kernel=%d limiter_steps=%d "
          "fallback_steps=%d oracle_limited_points=%d" % (
              precision, st["kernel"], st["limiter_steps"],
              st["fp64_fallback_steps"], int(lim.points().sum())),
          flush=True)
    assert st["kernel"] == expected_kernel(w, precision)
    assert st["active_points"] == 2000
    assert st["limiter_steps"] > 0
    if precision == 1:
        assert st["fp64_fallback_steps"] > 0
    check(got, ref, w.N, x, precision, "limiter-heavy", limited=lim, w=w)


@pytest.mark.parametrize("precision", [0, 1])
def test_limiter_heavy_full_size_sampled(precision):
    L = _lib()
    w = wl.config3_limiter_heavy()
    h = L.FsbmCoal.from_workload(w, precision=precision)
    N = _dev(w.N)
    h.step(N, _dev(w.p), w.dt, w.nsteps)
    torch.cuda.synchronize()
    idx = wl.sample_active(w, 256, seed=9)
    got = N[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    st = h.stats()
    h.close()
    sub = w.subset(idx)
    ref, x, lim = run_oracle(sub)
    print("limiter-heavy full precision=%d: kernel=%d limiter_steps=%d "
          "fallback_steps=%d" % (precision, st["kernel"],
                                 st["limiter_steps"],
                                 st["fp64_fallback_steps"]), flush=True)
    assert st["kernel"] == expected_kernel(w, precision)
    assert st["active_points"] == w.npoints
    assert lim.points().mean() > 0.5
    check(got, ref, sub.N, x, precision, "limiter-heavy-full", limited=lim,
          w=sub)
