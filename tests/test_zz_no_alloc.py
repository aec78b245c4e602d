"""fsbm_coal_step_noalloc (the entry point that allocates nothing: its
workspace is the library's static scratch block) against fsbm_coal_step on
the same inputs, through the C ABI.  Both run the same kernels over the same
workspace layout, so the bar is bit-for-bit equality; the second call of each
case is smaller than the first, so it runs over a block that still holds the
first call's contents."""

import ctypes

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl
from tests.parity import expected_kernel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _lib():
    from paper_2409_07232_amd import _lib as L
    return L


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _pair(w, precision, idx, stream=None):
    """(fsbm_coal_step result, fsbm_coal_step_noalloc result, stats of
    both, totals of both) on the points idx of w."""
    L = _lib()
    sub = w.subset(idx)
    ha = L.FsbmCoal.from_workload(w, precision=precision)
    hb = L.FsbmCoal.from_workload(w, precision=precision)
    Na, pa = _dev(sub.N), _dev(sub.p)
    Nb, pb = _dev(sub.N), _dev(sub.p)
    ha.step(Na, pa, w.dt, sub.nsteps, stream=stream)
    hb.step_noalloc(Nb, pb, w.dt, sub.nsteps, stream=stream)
    torch.cuda.synchronize()
    sa, sb = ha.stats(), hb.stats()
    ta = [t.cpu().numpy() for t in ha.totals()]
    tb = [t.cpu().numpy() for t in hb.totals()]
    torch.cuda.synchronize()
    out = Na.cpu().numpy(), Nb.cpu().numpy(), sa, sb, ta, tb
    ha.close()
    hb.close()
    return out


def _check(case, a, b, sa, sb, ta, tb):
    print("noalloc case %s: points %d, max |diff| %.3e" % (
        case, a.shape[0], float(np.abs(a - b).max()) if a.size else 0.0),
        flush=True)
    assert np.array_equal(a, b), case
    for k in ("active_points", "pair_evals", "limiter_steps",
              "fp64_fallback_steps", "exact_pair_evals"):
        assert sa[k] == sb[k], (case, k, sa[k], sb[k])
    for x, y in zip(ta, tb):
        assert np.array_equal(x, y), case


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_lane_kernels_two_calls(precision):
    """One species, 33 doubling bins (one point per lane): a 16 x 16 x 50
    thunderstorm patch, then a ragged subset of it."""
    w = wl.config2(nx=16, ny=16, nz=50, nsteps=30)
    first = np.arange(w.npoints)
    rng = np.random.default_rng(5)
    second = np.sort(rng.choice(w.npoints, 3001, replace=False))
    for tag, idx in (("lane-first", first), ("lane-second", second)):
        a, b, sa, sb, ta, tb = _pair(w, precision, idx)
        assert sa["kernel"] == 0
        _check("%s-p%d" % (tag, precision), a, b, sa, sb, ta, tb)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_multi_species_two_calls(precision):
    """Four species, 33 bins (FP32C: one point per lane for several
    species; FP64: one point per wave), then the refined 66-bin grid on
    fewer points (one point per wave): the second call reuses the block
    with another layout."""
    w3 = wl.config3(npoints=3000, nsteps=20)
    w4 = wl.config4(nbins=66, npoints=1200, nsteps=10)
    for tag, w in (("four-species", w3), ("refined66", w4)):
        a, b, sa, sb, ta, tb = _pair(w, precision, np.arange(w.npoints))
        assert sa["kernel"] == expected_kernel(w, precision)
        _check("%s-p%d" % (tag, precision), a, b, sa, sb, ta, tb)


def test_noalloc_on_a_stream_and_sequential_form():
    """A non-default stream, and the sequential form (in place, FP64)."""
    L = _lib()
    w = wl.config2(nx=8, ny=8, nz=50, nsteps=40)
    s = torch.cuda.Stream()
    a, b, sa, sb, ta, tb = _pair(w, 1, np.arange(w.npoints),
                                 stream=s)
    _check("stream", a, b, sa, sb, ta, tb)
    hs = [L.FsbmCoal.from_workload(w, precision=0,
                                   order=L.ORDER_SEQUENTIAL)
          for _ in range(2)]
    Na, Nb = _dev(w.N), _dev(w.N)
    p = _dev(w.p)
    hs[0].step(Na, p, w.dt, w.nsteps)
    hs[1].step_noalloc(Nb, p, w.dt, w.nsteps)
    torch.cuda.synchronize()
    assert np.array_equal(Na.cpu().numpy(), Nb.cpu().numpy())
    for h in hs:
        h.close()


def test_noalloc_rejects_a_call_beyond_the_block():
    """A call whose workspace exceeds the scratch block is refused before
    anything is enqueued, with the size in the message; the state is
    untouched and the next call within the limit runs."""
    L = _lib()
    w = wl.config2(nx=8, ny=8, nz=50, nsteps=5)
    # one species, 33 bins, lane kernels: 2 * 33 * 8 + 54 bytes per point
    P = SCRATCH_BYTES // (2 * 33 * 8) + 1000
    rng = np.random.default_rng(3)
    idx = rng.integers(0, w.npoints, P)
    N0 = np.ascontiguousarray(w.N[idx])
    N = _dev(N0)
    p = _dev(w.p[idx])
    h = L.FsbmCoal.from_workload(w, precision=1)
    with pytest.raises(L.FsbmError) as e:
        h.step_noalloc(N, p, w.dt, w.nsteps)
    assert e.value.code == L.FSBM_EUNSUPPORTED
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert np.array_equal(N.cpu().numpy(), N0)
    small = _dev(w.N)
    ref = _dev(w.N)
    h.step_noalloc(small, _dev(w.p), w.dt, w.nsteps)
    h2 = L.FsbmCoal.from_workload(w, precision=1)
    h2.step(ref, _dev(w.p), w.dt, w.nsteps)
    torch.cuda.synchronize()
    assert np.array_equal(small.cpu().numpy(), ref.cpu().numpy())
    h.close()
    h2.close()


def test_noalloc_no_op_and_argument_errors():
    L = _lib()
    lib = L.load()
    w = wl.config2(nx=4, ny=4, nz=50, nsteps=5)
    h = L.FsbmCoal.from_workload(w, precision=0)
    N = _dev(w.N)
    p = _dev(w.p)
    assert lib.fsbm_coal_step_noalloc(h.handle, N.data_ptr(), p.data_ptr(),
                                      0, 1.0, 3, None) == 0
    assert lib.fsbm_coal_step_noalloc(h.handle, N.data_ptr(), p.data_ptr(),
                                      w.npoints, 1.0, 0, None) == 0
    assert lib.fsbm_coal_step_noalloc(h.handle, N.data_ptr(), p.data_ptr(),
                                      w.npoints, -1.0, 3, None) == \
        L.FSBM_EINVAL
    assert lib.fsbm_coal_step_noalloc(None, N.data_ptr(), p.data_ptr(),
                                      w.npoints, 1.0, 3, None) == \
        L.FSBM_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(N.cpu().numpy(), w.N)
    h.close()
