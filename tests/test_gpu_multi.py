"""GPU parity of the one-point-per-lane kernels for several species (FP32C,
two to four species on the 33-bin doubling grid; points bucketed by pressure
bracket and by the species set they can hold during a call).

Bars as in the other parity tests: rel_bin 1e-5 (FP32C) against the FP64
oracle, relative mass drift 1e-10; launch shape and graph replay bit for
bit.
"""

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl
from tests.parity import check, expected_kernel, run_oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

MULTI = 3


def _lib():
    from paper_2409_07232_amd import _lib as L
    return L


def _run(w, precision=1, flags=0, steps_per_launch=0, stream=None, N=None,
         dt=None):
    L = _lib()
    h = L.FsbmCoal.from_workload(w, precision=precision, flags=flags,
                                 steps_per_launch=steps_per_launch)
    Nd = torch.from_numpy(np.array(w.N if N is None else N, copy=True)).to(
        "cuda")
    p = torch.from_numpy(np.array(w.p, copy=True)).to("cuda")
    h.step(Nd, p, w.dt if dt is None else dt, w.nsteps, stream=stream)
    torch.cuda.synchronize()
    out = Nd.cpu().numpy()
    st = h.stats()
    h.close()
    return out, st


def _every_species_set(npoints_per_set=70, nsteps=40):
    """The four-species workload with every subset of the four species
    present at some points (points of the empty set are dry): each species
    set closes under the product map to one of the kernel's buckets (ice
    alone makes snow), ragged counts per bucket."""
    w = wl.config3(npoints=16 * npoints_per_set, nsteps=nsteps)
    N = np.array(w.N, copy=True)
    rng = np.random.default_rng(7)
    # species present in w where drawn; fill every species first so that a
    # pattern can switch any of them on
    full = wl.config3(npoints=16 * npoints_per_set, nsteps=nsteps)
    donor = np.roll(full.N, 1, axis=0)
    for s in range(4):
        empty = N[:, s, :].sum(axis=1) == 0.0
        N[empty, s, :] = donor[empty, s, :]
        still = N[:, s, :].sum(axis=1) == 0.0
        N[still, s, :] = full.N[still, 0, :] * (0.1 + s)
    masks = rng.permutation(np.arange(16 * npoints_per_set) % 16)
    for s in range(4):
        N[(masks >> s) & 1 == 0, s, :] = 0.0
    w.N = N
    return w, masks


def test_multi_four_species_against_oracle():
    w = wl.config3(npoints=2000, nsteps=40)
    ref, x, lim = run_oracle(w)
    got, st = _run(w)
    assert st["kernel"] == MULTI == expected_kernel(w, 1)
    assert st["active_points"] == 2000
    check(got, ref, w.N, x, 1, "multi4", limited=lim, w=w)


def test_multi_every_species_set():
    """All 15 nonempty species sets (NS = 1..4 after closure) and dry
    points in one call."""
    w, masks = _every_species_set()
    ref, x, lim = run_oracle(w)
    got, st = _run(w)
    dry = masks == 0
    assert st["kernel"] == MULTI
    assert st["active_points"] == int((~dry).sum())
    assert np.array_equal(got[dry], w.N[dry])
    # species that no collision of the point's set can produce stay empty
    check(got, ref, w.N, x, 1, "multi-sets", limited=lim, w=w)
    prod = w.product
    for m in range(1, 16):
        c = m
        while True:
            c2 = c
            for a in range(4):
                for b in range(4):
                    if (c >> a) & 1 and (c >> b) & 1:
                        c2 |= 1 << int(prod[a, b])
            if c2 == c:
                break
            c = c2
        sel = masks == m
        for s in range(4):
            if not (c >> s) & 1:
                assert np.all(got[sel, s, :] == 0.0), (m, s)


@pytest.mark.parametrize("nspecies", [2, 3])
def test_multi_other_species_counts(nspecies):
    """Two and three species with a product map max(a, b) and distinct
    fall-speed laws for every pair table; one pressure level too."""
    rng = np.random.default_rng(30 + nspecies)
    B = 33
    rho = tuple([1.0, 0.4, 0.9][:nspecies])
    beta = tuple([0.8, 0.6, 0.3][:nspecies])
    rbar = tuple([10e-4, 300e-4, 100e-4][:nspecies])
    for levels in (wl.P_LEVELS_3, np.array([800.0])):
        tables = wl.gravitational_tables(B, 1, rho, beta,
                                         wl.multi_species_vcoef(beta),
                                         levels)
        prod = np.maximum.outer(np.arange(nspecies),
                                np.arange(nspecies)).astype(np.int32)
        x = wl.bin_masses(B)
        npts = 333
        present = rng.random((npts, nspecies)) < 0.6
        present[:, 0] |= ~present.any(axis=1)
        N = wl._multi_species_states(
            rng, x, rho, rbar, tuple([(0.05, 1.0)] * nspecies), present,
            npts, ((0, 5), (15, 32)))
        p = rng.uniform(500.0, 1000.0, npts)
        w = wl.Workload("custom", B, nspecies, 1, tables, levels.copy(),
                        prod, N, p, 2.0, 30)
        ref, x, lim = run_oracle(w)
        got, st = _run(w)
        assert st["kernel"] == MULTI
        check(got, ref, w.N, x, 1, "multi%d-L%d" % (nspecies, len(levels)),
              limited=lim, w=w)


def test_multi_forced_limiter():
    """A time step long enough that many points over-demand a bin: those
    points finish the call on the exact FP64 path (limiter included)."""
    w = wl.config3(npoints=640, nsteps=6)
    ref, x, lim = run_oracle(w, dt=300.0)
    got, st = _run(w, dt=300.0)
    assert st["kernel"] == MULTI
    assert st["fp64_fallback_steps"] > 0
    assert lim.sum() > 0
    check(got, ref, w.N, x, 1, "multi-limiter", limited=lim, w=w,
          dt=300.0)


@pytest.mark.parametrize("npts", [1, 63, 65, 130])
def test_multi_ragged_point_counts(npts):
    w = wl.config3(npoints=400, nsteps=15)
    idx = np.sort(np.random.default_rng(npts).choice(400, npts,
                                                     replace=False))
    sub = w.subset(idx)
    ref, x, lim = run_oracle(sub)
    got, st = _run(sub)
    assert st["kernel"] == MULTI
    check(got, ref, sub.N, x, 1, "multi-ragged%d" % npts, limited=lim,
          w=sub)


def test_multi_launch_shape_and_graph_replay():
    """Steps per launch and hipGraph replays do not change a bit."""
    L = _lib()
    w, _ = _every_species_set(npoints_per_set=40, nsteps=23)
    base, _ = _run(w, flags=L.FLAG_NO_GRAPH)
    for spl in (1, 7, 23):
        got, st = _run(w, flags=L.FLAG_NO_GRAPH, steps_per_launch=spl)
        assert st["steps_per_launch"] == spl
        assert np.array_equal(got, base), spl
    h = L.FsbmCoal.from_workload(w, precision=1)
    s = torch.cuda.Stream()
    p = torch.from_numpy(np.array(w.p, copy=True)).to("cuda")
    N = torch.empty((w.npoints, 4, 33), dtype=torch.float64, device="cuda")
    N0 = torch.from_numpy(np.array(w.N, copy=True)).to("cuda")
    for rep in range(3):
        N.copy_(N0)
        torch.cuda.synchronize()
        h.step(N, p, w.dt, w.nsteps, stream=s)
        s.synchronize()
        assert np.array_equal(N.cpu().numpy(), base), rep
    assert h.stats()["graph_captures"] == 1
    h.close()


def test_multi_needs_fp32c_and_the_doubling_grid():
    """FP64 handles and FORCE_WAVE stay on the one-point-per-wave kernel;
    both agree with the multi-species kernel within the FP32C bar."""
    L = _lib()
    w = wl.config3(npoints=300, nsteps=20)
    ref, x, lim = run_oracle(w)
    got64, st64 = _run(w, precision=0)
    assert st64["kernel"] == 1
    check(got64, ref, w.N, x, 0, "multi-fp64", limited=lim, w=w)
    gotw, stw = _run(w, precision=1, flags=L.FLAG_FORCE_WAVE)
    assert stw["kernel"] == 1
    check(gotw, ref, w.N, x, 1, "multi-forcewave", limited=lim, w=w)
