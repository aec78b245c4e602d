"""GPU parity of FSBM's per-point gates and species structure.

* Temperature gates of the loop over grid points (Sec. III, main-loop
  listing): collisions only where the previous temperature exceeds
  193.15 K and the current one 223.15 K.  fsbm_coal_step_gated against the
  oracle's gated run; gated points bitwise unchanged; points exactly at a
  threshold are gated; the totals of gated points report their mass.
* Ice-crystal habits (the habit dimension of FSBM's crystal arrays,
  Sec. VI-C): seven species (liquid, columns, plates, dendrites, snow,
  graupel, hail) with 28 pair kernels on 33 bins, run by the one-point-per-
  wave kernel, against the oracle.

Bars as in the other parity tests: rel_bin 1e-12 (FP64) / 1e-5 (FP32C),
relative mass drift 1e-10.
"""

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl
from tests.parity import check, expected_kernel, model_of, run_oracle, Limited

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2409_07232_amd import _lib as L
    return L


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _oracle_gated(w, t_old, t_now):
    om = model_of(w)
    Nr = np.array(w.N, copy=True)
    res = om.run(Nr, w.p, w.dt, w.nsteps, t_old=t_old, t_now=t_now,
                 totals=True)
    return Nr, om.grid(), Limited(res["limiter_per_point"],
                                  res["limited_bins"]), res


@pytest.mark.parametrize("precision", [0, 1])
def test_gated_thunderstorm_patch(precision):
    """16 x 16 x 50 thunderstorm patch, temperatures on both sides of both
    thresholds, 60 steps (one point per lane)."""
    L = _lib()
    w = wl.config2(nx=16, ny=16, nz=50, nsteps=60)
    t_old, t_now = wl.temperatures(w.npoints, seed=1)
    # a few points exactly at a threshold, and a NaN: all gated
    wet = np.flatnonzero(w.cloudy())
    t_now[wet[:3]] = 223.15
    t_old[wet[3:6]] = 193.15
    t_now[wet[6]] = np.nan
    ref, x, lim, res = _oracle_gated(w, t_old, t_now)
    on = (t_old > 193.15) & (t_now > 223.15) & w.cloudy()
    assert 100 < on.sum() < w.cloudy().sum() - 100
    h = L.FsbmCoal.from_workload(w, precision=precision)
    N = _dev(w.N)
    h.step_gated(N, _dev(w.p), _dev(t_old), _dev(t_now), w.dt, w.nsteps)
    torch.cuda.synchronize()
    got = N.cpu().numpy()
    st = h.stats()
    mb, ma, nb, na = [t.cpu().numpy() for t in h.totals()]
    print("gated patch precision=%d: %d of %d cloudy points pass the gates"
          % (precision, int(on.sum()), int(w.cloudy().sum())), flush=True)
    assert st["active_points"] == int(on.sum())
    assert np.array_equal(got[~on], w.N[~on])
    check(got, ref, w.N, x, precision, "gated", limited=lim, w=w)
    # totals: gated wet points keep mass and number before = after, equal
    # to the oracle's FP64 totals of the unchanged state
    gated_wet = w.cloudy() & ~on
    np.testing.assert_allclose(mb[gated_wet], res["mass_before"][gated_wet],
                               rtol=1e-13)
    assert np.array_equal(mb[gated_wet], ma[gated_wet])
    assert np.array_equal(nb[gated_wet], na[gated_wet])
    np.testing.assert_allclose(ma[on], res["mass_after"][on], rtol=1e-10)
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_gated_equals_ungated_where_warm(precision):
    """Four species (one point per wave): with every point warm the gated
    call equals the plain one bit for bit; with one array NULL only the
    other test applies."""
    L = _lib()
    w = wl.config3(npoints=2000, nsteps=15)
    h = L.FsbmCoal.from_workload(w, precision=precision)
    warm = np.full(w.npoints, 280.0)
    Na, Nb = _dev(w.N), _dev(w.N)
    p = _dev(w.p)
    h.step(Na, p, w.dt, w.nsteps)
    h.step_gated(Nb, p, _dev(warm), _dev(warm), w.dt, w.nsteps)
    torch.cuda.synchronize()
    assert np.array_equal(Na.cpu().numpy(), Nb.cpu().numpy())
    # only t_now given: the t_old test passes everywhere
    t_old, t_now = wl.temperatures(w.npoints, seed=2)
    ref, x, lim, _ = _oracle_gated(w, None, t_now)
    Nc = _dev(w.N)
    h.step_gated(Nc, p, None, _dev(t_now), w.dt, w.nsteps)
    torch.cuda.synchronize()
    got = Nc.cpu().numpy()
    off = ~(t_now > 223.15)
    assert np.array_equal(got[off], w.N[off])
    check(got, ref, w.N, x, precision, "gated-now-only", limited=lim, w=w)
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_seven_species_habits(precision):
    """Seven species with three ice-crystal habits, 33 bins, 28 pair
    kernels, 1500 points, 40 steps of 2 s."""
    L = _lib()
    w = wl.config_habits(npoints=1500, nsteps=40)
    ref, x, lim = run_oracle(w)
    h = L.FsbmCoal.from_workload(w, precision=precision)
    N = _dev(w.N)
    h.step(N, _dev(w.p), w.dt, w.nsteps)
    torch.cuda.synchronize()
    got = N.cpu().numpy()
    st = h.stats()
    assert st["kernel"] == 1
    assert st["active_points"] == int(w.cloudy().sum())
    check(got, ref, w.N, x, precision, "habits7", limited=lim, w=w)
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_seven_species_full_size_sampled(precision):
    """The seven-species workload at 2^18 points and 100 steps, as one
    call; 256 seeded points checked against the oracle."""
    L = _lib()
    w = wl.config_habits()
    h = L.FsbmCoal.from_workload(w, precision=precision)
    N = _dev(w.N)
    h.step(N, _dev(w.p), w.dt, w.nsteps)
    torch.cuda.synchronize()
    idx = wl.sample_active(w, 256, seed=4)
    got = N[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    sub = w.subset(idx)
    ref, x, lim = run_oracle(sub)
    st = h.stats()
    print("habits7 full precision=%d: limiter_steps=%d fallback_steps=%d"
          % (precision, st["limiter_steps"], st["fp64_fallback_steps"]),
          flush=True)
    check(got, ref, sub.N, x, precision, "habits7-full", limited=lim, w=sub)
    h.close()
