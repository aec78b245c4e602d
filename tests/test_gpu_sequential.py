"""GPU parity of the sequential (in-place) form of Bott's flux method: the
one-point-per-lane sequential kernel through the C ABI against the oracle's
sequential mode, FP64 only.

Bar: rel_bin <= 1e-12 (floor 1e-9 M_tot; 1e-3 M_tot for points at which the
oracle capped a pair, since a cap empties a bin by cancellation exactly as
the limiter does), mass drift <= 1e-10, positivity; results independent of
the launch shape and identical over graph replays, bit for bit.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl
from tests.parity import DRIFT, check, run_oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lib():
    from paper_2409_07232_amd import _lib as L
    return L


def seq_handle(w, **kw):
    L = _lib()
    return L.FsbmCoal.from_workload(w, precision=L.FSBM_FP64,
                                    order=L.ORDER_SEQUENTIAL, **kw)


def run_gpu(w, N=None, p=None, dt=None, nsteps=None, handle=None, **kw):
    h = handle or seq_handle(w, **kw)
    Nd = torch.from_numpy(np.ascontiguousarray(w.N if N is None else N)).to(
        "cuda")
    pd = torch.from_numpy(np.ascontiguousarray(w.p if p is None else p)).to(
        "cuda")
    h.step(Nd, pd, w.dt if dt is None else dt,
           w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    return Nd.cpu().numpy(), h.stats(), h


def test_three_bin_worked_example_exact():
    """The hand-worked 3-bin step (exact binary fractions) on the GPU."""
    L = _lib()
    with open(os.path.join(GOLDEN, "sequential_worked_examples.json")) as f:
        case = [c for c in json.load(f)["cases"] if c["nbins"] == 3][0]
    B = 3
    h = L.FsbmCoal(B, 1, np.full((1, 1, B, B), case["K"]), np.array([1000.0]),
                   x1_g=1.0, order=L.ORDER_SEQUENTIAL)
    # the same point in 64 lanes plus ragged padding
    N = np.tile(np.array(case["N"])[None, None, :], (70, 1, 1))
    Nd = torch.from_numpy(N).to("cuda")
    pd = torch.full((70,), 1000.0, dtype=torch.float64, device="cuda")
    h.step(Nd, pd, case["dt"], 1)
    torch.cuda.synchronize()
    M = Nd.cpu().numpy()[:, 0, :] * np.array([1.0, 2.0, 4.0])
    want = [Fraction(v) for v in case["M_after"]]
    for row in M:
        assert [Fraction(float(v)) for v in row] == want
    assert h.stats()["kernel"] == 2


@pytest.mark.parametrize("dt", [0.5, 3.0, 100.0])
def test_unit_grid_cases(dt):
    """Small grids with a constant kernel, caps off and on."""
    L = _lib()
    B = 8
    t = np.full((1, 1, B, B), 0.25)
    rng = np.random.default_rng(11)
    N = rng.uniform(0.0, 2.0, (130, 1, B))
    N[:, :, 5:] = 0.0
    N[::7] = 0.0
    w = wl.Workload("unit8", B, 1, 1, t, np.array([1000.0]),
                    np.zeros((1, 1), np.int32), N, np.full(130, 1000.0), dt,
                    3, x1_g=1.0)
    ref, x, lim = run_oracle(w, order=1)
    h = L.FsbmCoal(B, 1, t, np.array([1000.0]), x1_g=1.0,
                   order=L.ORDER_SEQUENTIAL)
    got, st, _ = run_gpu(w, handle=h)
    check(got, ref, N, x, 0, "unit%g" % dt, limited=lim)
    if dt > 50.0:
        assert lim.sum() > 0 and st["limiter_steps"] > 0


def test_golovin_full_run():
    w = wl.config1(npoints=64)
    ref, x, lim = run_oracle(w.subset(np.arange(1)), order=1)
    got, st, _ = run_gpu(w)
    check(got, np.repeat(ref, 64, axis=0), w.N, x, 0, "seq-golovin",
          limited=lim.repeat(64))
    assert st["active_points"] == 64


def test_thunderstorm_patch_small():
    w = wl.config2(nx=16, ny=16, nz=50)
    ref, x, lim = run_oracle(w, order=1)
    got, st, _ = run_gpu(w)
    dry = ~w.cloudy()
    assert np.array_equal(got[dry], w.N[dry])
    check(got, ref, w.N, x, 0, "seq-patch16", limited=lim)
    assert st["active_points"] == int((~dry).sum())
    assert st["limiter_steps"] == 0 and lim.sum() == 0


@pytest.mark.parametrize("npts", [1, 63, 65, 130])
def test_ragged_point_counts(npts):
    w = wl.config2(nx=8, ny=8, nz=50)
    idx = np.sort(np.random.default_rng(npts).choice(w.npoints, npts,
                                                     replace=False))
    sub = w.subset(idx)
    sub.nsteps = 20
    ref, x, lim = run_oracle(sub, order=1)
    got, _, _ = run_gpu(sub)
    check(got, ref, sub.N, x, 0, "seq-ragged%d" % npts, limited=lim)


def test_caps_at_huge_time_step():
    w = wl.config2(nx=8, ny=8, nz=50)
    sub = w.subset(wl.sample_active(w, 96))
    ref, x, lim = run_oracle(sub, dt=4000.0, nsteps=3, order=1)
    got, st, _ = run_gpu(sub, dt=4000.0, nsteps=3)
    assert lim.sum() > 0 and st["limiter_steps"] > 0
    # A cap leaves bin i with M_i - (M_i / x_i) x_i: zero, or a residue of
    # about one ulp of either sign depending on rounding; a positive residue
    # is still active and caps the next pairs of the row again.  The counts
    # therefore agree only in size, while the masses agree to the bar.
    ratio = st["limiter_steps"] / float(lim.sum())
    print("capped pairs gpu %d oracle %d" % (st["limiter_steps"], lim.sum()))
    assert 0.5 <= ratio <= 2.0
    check(got, ref, sub.N, x, 0, "seq-caps", limited=lim)


def test_launch_shape_graph_replay_and_determinism():
    w = wl.config2(nx=8, ny=8, nz=50)
    w.nsteps = 30
    L = _lib()
    base, _, _ = run_gpu(w, flags=L.FLAG_NO_GRAPH)
    for spl in (1, 7, 30):
        h = seq_handle(w, flags=L.FLAG_NO_GRAPH, steps_per_launch=spl)
        got, _, _ = run_gpu(w, handle=h)
        assert np.array_equal(got, base), spl
    s = torch.cuda.Stream()
    h = seq_handle(w)
    p = torch.from_numpy(w.p.copy()).to("cuda")
    N0 = torch.from_numpy(w.N.copy()).to("cuda")
    N = torch.empty_like(N0)
    for rep in range(3):          # capture once, replay twice
        with torch.cuda.stream(s):
            N.copy_(N0)
            h.step(N, p, w.dt, w.nsteps, stream=s)
        s.synchronize()
        assert np.array_equal(N.cpu().numpy(), base)


def test_autotune_keeps_results(tmp_path, monkeypatch):
    monkeypatch.setenv("FSBM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = wl.config2(nx=8, ny=8, nz=50)
    w.nsteps = 20
    L = _lib()
    base, _, _ = run_gpu(w, flags=L.FLAG_NO_GRAPH)
    h = seq_handle(w)
    h.tune(4096)
    got, st, _ = run_gpu(w, handle=h)
    assert np.array_equal(got, base)
    print("tuned", st["steps_per_launch"], st["waves_per_block"], flush=True)


def test_unsupported_shapes_rejected():
    L = _lib()
    for w, prec in ((wl.config2(nx=4, ny=4, nz=50), L.FSBM_FP32C),
                    (wl.config3(npoints=64), L.FSBM_FP64),
                    (wl.config4(nbins=66, npoints=64), L.FSBM_FP64)):
        with pytest.raises(L.FsbmError) as e:
            L.FsbmCoal.from_workload(w, precision=prec,
                                     order=L.ORDER_SEQUENTIAL)
        assert e.value.code == L.FSBM_EUNSUPPORTED


def test_full_size_thunderstorm_sampled():
    """The benchmark workload at full size (256 x 256 x 50, 100 steps of
    2 s) in the sequential form; 256 sampled cloudy points against the
    oracle, conservation and number decrease on every point."""
    w = wl.config2()
    h = seq_handle(w)
    N = torch.from_numpy(w.N).to("cuda")
    p = torch.from_numpy(w.p).to("cuda")
    h.step(N, p, w.dt, w.nsteps)
    torch.cuda.synchronize()
    mb, ma, nb, na = [t.cpu().numpy() for t in h.totals()]
    cl = mb > 0
    assert np.max(np.abs(ma[cl] - mb[cl]) / mb[cl]) <= DRIFT
    assert np.all(na <= nb * (1 + 1e-12))
    idx = wl.sample_active(w, 256, seed=7)
    got = N[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    assert np.all(got >= 0)
    sub = w.subset(idx)
    ref, x, lim = run_oracle(sub, order=1)
    check(got, ref, sub.N, x, 0, "seq-full-sampled", limited=lim)


@pytest.mark.parametrize("nbins", [3, 8, 16, 40])
def test_every_bin_count(nbins):
    """Each bin count the sequential kernel is built for (Golovin runs,
    points varied by a seeded scale and per-bin noise, 70 points)."""
    w = wl.config1(npoints=70, nbins=nbins, nsteps=40, dt=2.0)
    rng = np.random.default_rng(5)
    w.N = np.ascontiguousarray(w.N * np.exp(rng.uniform(-1, 1, (70, 1, 1))) *
                               rng.uniform(0.8, 1.2, w.N.shape))
    ref, x, lim = run_oracle(w, order=1)
    got, st, _ = run_gpu(w)
    assert st["kernel"] == 2
    check(got, ref, w.N, x, 0, "seq%d" % nbins, limited=lim)


def test_degenerate_calls():
    L = _lib()
    w = wl.config2(nx=8, ny=8, nz=50)
    h = seq_handle(w)
    got, _, _ = run_gpu(w, nsteps=0, handle=h)
    assert np.array_equal(got, w.N)
    dry = np.zeros_like(w.N)
    got, st, _ = run_gpu(w, N=dry, handle=h)
    assert np.array_equal(got, dry)
    assert st["active_points"] == 0
    Nd = torch.zeros((0, 1, w.nbins), dtype=torch.float64, device="cuda")
    pd = torch.zeros((0,), dtype=torch.float64, device="cuda")
    h.step(Nd, pd, 2.0, 5)
    with pytest.raises(L.FsbmError) as e:
        Nd = torch.from_numpy(w.N.copy()).to("cuda")
        pd = torch.from_numpy(w.p.copy()).to("cuda")
        h.step(Nd, pd, -1.0, 5)
    assert e.value.code == L.FSBM_EINVAL
