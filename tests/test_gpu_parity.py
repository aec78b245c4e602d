"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (rel_bin: max over points, species, bins of |dM| / max(|M_ref|,
1e-9 M_tot)): FP64 path 1e-12, FP32C path 1e-5; relative per-point mass
drift 1e-10 for both.
"""

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl
from tests.parity import DRIFT, check, expected_kernel, run_oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2409_07232_amd import _lib as L
    return L


def run_gpu(w, precision, N=None, p=None, dt=None, nsteps=None, flags=0,
            stream=None, handle=None):
    L = _lib()
    h = handle or L.FsbmCoal.from_workload(w, precision=precision,
                                           flags=flags)
    Nd = torch.from_numpy(np.ascontiguousarray(w.N if N is None else N)).to(
        "cuda")
    pd = torch.from_numpy(np.ascontiguousarray(w.p if p is None else p)).to(
        "cuda")
    h.step(Nd, pd, w.dt if dt is None else dt,
           w.nsteps if nsteps is None else nsteps, stream=stream)
    torch.cuda.synchronize()
    out = Nd.cpu().numpy()
    st = h.stats()
    return out, st, h


@pytest.mark.parametrize("precision", [0, 1])
def test_golovin_full_run(precision):
    """64 identical points, 33 bins, Golovin kernel, dt 1 s x 1800 steps."""
    w = wl.config1(npoints=64)
    ref, x, lim = run_oracle(w.subset(np.arange(1)))
    got, st, _ = run_gpu(w, precision)
    check(got, np.repeat(ref, 64, axis=0), w.N, x, precision, "golovin",
          limited=lim.repeat(64))
    assert st["active_points"] == 64
    assert st["limiter_steps"] == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_thunderstorm_patch_small(precision):
    """Config-2 recipe on a 16 x 16 x 50 patch (about 1900 cloudy points,
    several waves per pressure bracket and ragged tails), 100 steps."""
    w = wl.config2(nx=16, ny=16, nz=50)
    ref, x, lim = run_oracle(w)
    got, st, _ = run_gpu(w, precision)
    dry = ~w.cloudy()
    assert np.array_equal(got[dry], w.N[dry])
    check(got, ref, w.N, x, precision, "patch16", limited=lim, w=w)
    assert st["active_points"] == int((~dry).sum())


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("npts", [1, 63, 65, 130])
def test_ragged_point_counts(precision, npts):
    w = wl.config2(nx=8, ny=8, nz=50)
    idx = np.sort(np.random.default_rng(npts).choice(w.npoints, npts,
                                                     replace=False))
    sub = w.subset(idx)
    sub.nsteps = 20
    ref, x, lim = run_oracle(sub)
    got, _, _ = run_gpu(sub, precision)
    check(got, ref, sub.N, x, precision, "ragged%d" % npts, limited=lim,
          w=sub)


@pytest.mark.parametrize("precision", [0, 1])
def test_degenerate_calls(precision):
    w = wl.config2(nx=8, ny=8, nz=50)
    L = _lib()
    h = L.FsbmCoal.from_workload(w, precision=precision)
    # zero steps: identity, bitwise
    got, _, _ = run_gpu(w, precision, nsteps=0, handle=h)
    assert np.array_equal(got, w.N)
    # all points dry: untouched, bitwise
    dry = np.zeros_like(w.N)
    got, st, _ = run_gpu(w, precision, N=dry, handle=h)
    assert np.array_equal(got, dry)
    assert st["active_points"] == 0
    # zero points: accepted no-op
    Nd = torch.zeros((0, 1, w.nbins), dtype=torch.float64, device="cuda")
    pd = torch.zeros((0,), dtype=torch.float64, device="cuda")
    h.step(Nd, pd, 2.0, 5)
    # invalid arguments are rejected with EINVAL, the state untouched
    Nd = torch.from_numpy(w.N.copy()).to("cuda")
    pd = torch.from_numpy(w.p.copy()).to("cuda")
    for dt, n in ((-1.0, 5), (0.0, 5), (float("nan"), 5),
                  (float("inf"), 5), (2.0, -1)):
        with pytest.raises(L.FsbmError) as e:
            h.step(Nd, pd, dt, n)
        assert e.value.code == L.FSBM_EINVAL
    lib = L.load()
    assert lib.fsbm_coal_step(h.handle, Nd.data_ptr(), pd.data_ptr(), -1,
                              2.0, 5, None) == L.FSBM_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(Nd.cpu().numpy(), w.N)


@pytest.mark.parametrize("precision", [0, 1])
def test_forced_limiter(precision):
    """A huge time step over-demands bins: the limiter path must match the
    oracle and keep mass and positivity (limited points are judged with the
    limiter floor of the parity helpers)."""
    w = wl.config2(nx=8, ny=8, nz=50)
    sub = w.subset(wl.sample_active(w, 96))
    ref, x, lim = run_oracle(sub, dt=4000.0, nsteps=3)
    got, st, _ = run_gpu(sub, precision, dt=4000.0, nsteps=3)
    assert st["limiter_steps"] > 0 and lim.sum() > 0
    check(got, ref, sub.N, x, precision, "limiter", limited=lim)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_and_determinism(precision):
    w = wl.config2(nx=8, ny=8, nz=50)
    w.nsteps = 30
    L = _lib()
    s = torch.cuda.Stream()
    h = L.FsbmCoal.from_workload(w, precision=precision)
    p = torch.from_numpy(w.p.copy()).to("cuda")
    outs = []
    N = torch.empty((w.npoints, 1, w.nbins), dtype=torch.float64,
                    device="cuda")
    N0 = torch.from_numpy(w.N.copy()).to("cuda")
    for rep in range(3):          # capture once, replay twice
        with torch.cuda.stream(s):
            N.copy_(N0)
            h.step(N, p, w.dt, w.nsteps, stream=s)
        s.synchronize()
        outs.append(N.cpu().numpy())
    hd = L.FsbmCoal.from_workload(w, precision=precision,
                                  flags=L.FLAG_NO_GRAPH)
    direct, _, _ = run_gpu(w, precision, handle=hd)
    for o in outs:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(outs[0], direct)


@pytest.mark.parametrize("precision", [0, 1])
def test_totals_and_pair_count(precision):
    w = wl.config2(nx=8, ny=8, nz=50)
    got, st, h = run_gpu(w, precision, nsteps=1)
    x = wl.bin_masses(w.nbins)
    mb, ma, nb, na = [t.cpu().numpy() for t in h.totals()]
    m0 = (w.N[:, 0, :] * x).sum(axis=1)
    m1 = (got[:, 0, :] * x).sum(axis=1)
    assert np.allclose(mb, m0, rtol=1e-14, atol=0)
    assert np.allclose(ma, m1, rtol=1e-14, atol=0)
    assert np.allclose(nb, w.N.sum(axis=(1, 2)), rtol=1e-14, atol=0)
    assert np.all(na <= nb * (1 + 1e-12))
    # pairs of one step: both bins active (M >= theta M_tot), target on
    # the grid and a kernel entry nonzero at some level; the gravitational
    # kernel is zero on the diagonal (equal fall speeds), so no self pair
    M = w.N[:, 0, :] * x
    tot = M.sum(axis=1, keepdims=True)
    act = (M > 0) & (M >= 1e-30 * tot)
    B = w.nbins
    i, j = np.triu_indices(B)
    on_grid = (i != j) | (j < B - 1)      # (B-1, B-1) leaves the grid
    nonzero = np.any(w.tables[0][:, i, j] != 0.0, axis=0)
    assert not nonzero[i == j].any()
    keep = on_grid & nonzero
    want = int((act[:, i[keep]] & act[:, j[keep]]).sum())
    n = act.sum(axis=1)
    assert want == int((n * (n - 1) // 2).sum())
    assert st["pair_evals"] == want


@pytest.mark.parametrize("precision", [1, 0])
def test_full_size_thunderstorm_sampled(precision):
    """The benchmark workload at full size (256 x 256 x 50 points, 100 steps
    of 2 s) in the benchmark's launch configuration; 256 sampled cloudy
    points checked against the oracle, conservation and positivity checked
    on every point through the FP64 totals."""
    w = wl.config2()
    L = _lib()
    h = L.FsbmCoal.from_workload(w, precision=precision)
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
    ref, x, lim = run_oracle(sub)
    check(got, ref, sub.N, x, precision, "full-sampled", limited=lim,
          w=sub)
    st = h.stats()
    assert st["active_points"] == int(cl.sum())


def _varied_golovin(nbins, npts=70, nsteps=40, seed=5):
    """Golovin runs on a B-bin doubling grid, points varied by a seeded
    overall scale and per-bin noise (ragged count: one full wave + 6)."""
    w = wl.config1(npoints=npts, nbins=nbins, nsteps=nsteps, dt=2.0)
    rng = np.random.default_rng(seed)
    scale = np.exp(rng.uniform(-1.0, 1.0, (npts, 1, 1)))
    noise = rng.uniform(0.8, 1.2, w.N.shape)
    w.N = np.ascontiguousarray(w.N * scale * noise)
    return w


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nbins", [3, 8, 16, 40])
def test_every_lane_bin_count(precision, nbins):
    """Each bin count the one-point-per-lane kernels are built for."""
    w = _varied_golovin(nbins)
    ref, x, lim = run_oracle(w)
    got, st, _ = run_gpu(w, precision)
    assert st["kernel"] == 0
    check(got, ref, w.N, x, precision, "lane%d" % nbins, limited=lim, w=w)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["lane", "wave"])
def test_handle_reused_on_fewer_points(precision, kind):
    """A handle's workspace is sized by the largest call so far; a later
    call on fewer points (compaction blocks past its last point, a ragged
    tail inside a block) must equal a fresh handle's result bit for bit
    and the oracle to the bar."""
    L = _lib()
    if kind == "lane":
        w = wl.config2(nx=8, ny=8, nz=50)
    else:
        # four species: one point per wave (FP64) or, FP32C, one point per
        # lane for several species
        w = wl.config3(npoints=3000)
    w.nsteps = 10
    h = L.FsbmCoal.from_workload(w, precision=precision)
    run_gpu(w, precision, handle=h)
    idx = np.sort(np.random.default_rng(3).choice(w.npoints, 301,
                                                  replace=False))
    sub = w.subset(idx)
    got, st, _ = run_gpu(sub, precision, handle=h)
    fresh, _, _ = run_gpu(sub, precision)
    assert np.array_equal(got, fresh)
    assert st["kernel"] == expected_kernel(w, precision)
    ref, x, lim = run_oracle(sub)
    check(got, ref, sub.N, x, precision, "reuse-" + kind, limited=lim,
          w=sub)


@pytest.mark.parametrize("bad", [-1e-3, np.nan, np.inf])
def test_debug_checks_refuse_invalid_states(bad):
    """With FSBM_FLAG_DEBUG_CHECKS a state holding a negative, NaN or
    infinite number is refused with FSBM_EDOMAIN before any step runs (the
    caller's array is left as it was); a valid state steps exactly as
    without the flag."""
    L = _lib()
    w = wl.config2(nx=8, ny=8, nz=50)
    w.nsteps = 5
    h = L.FsbmCoal.from_workload(w, precision=1, flags=L.FLAG_DEBUG_CHECKS)
    checked, _, _ = run_gpu(w, 1, handle=h)
    plain, _, _ = run_gpu(w, 1)
    assert np.array_equal(checked, plain)
    N = w.N.copy()
    pt = np.flatnonzero(w.cloudy())[3]
    N[pt, 0, 5] = bad
    Nd = torch.from_numpy(N.copy()).to("cuda")
    pd = torch.from_numpy(w.p.copy()).to("cuda")
    with pytest.raises(L.FsbmError) as e:
        h.step(Nd, pd, w.dt, w.nsteps)
    assert e.value.code == L.FSBM_EDOMAIN
    torch.cuda.synchronize()
    assert np.array_equal(Nd.cpu().numpy(), N, equal_nan=True)
