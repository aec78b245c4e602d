"""Pins of the oracle's sequential (in-place) form of Bott's flux method.

The sequential form takes the bin pairs one after another and moves mass in
place, so each pair sees what the pairs before it did (Bott's original
update; the simultaneous form of the main oracle is its Jacobi
counterpart).  It is pinned against:
  - hand-worked steps in exact binary fractions (tests/golden/), which fix
    the pair order, the in-place reads, the self-pair factor, the cap and
    the flux of the merged mass;
  - the simultaneous oracle (itself pinned in test_oracle_pins.py): both
    integrate the same collection equation, so one step differs by O(dt^2)
    and runs over a fixed time converge to each other as O(dt);
  - the Golovin closed form with its refinement ladder;
  - conservation, positivity and number decrease at any time step.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import compare
from paper_2409_07232_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def model_of(w, order):
    return oracle.OracleModel(w.nbins, w.nspecies, w.tables, w.p_levels,
                              w.product, x1_g=w.x1_g, s=w.s, theta=w.theta,
                              order=order)


def unit_grid_model(B, K, order=1):
    """x_k = 2^k g, one pressure level, constant kernel K."""
    return oracle.OracleModel(B, 1, np.full((1, 1, B, B), K),
                              np.array([1000.0]), np.zeros((1, 1), np.int32),
                              x1_g=1.0, order=order)


def _cases():
    with open(os.path.join(GOLDEN, "sequential_worked_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_worked_examples_exact(case):
    B = case["nbins"]
    om = unit_grid_model(B, case["K"])
    N = np.array([[case["N"]]], dtype=np.float64)
    r = om.run(N, np.array([1000.0]), case["dt"], 1)
    M = N[0, 0] * om.grid()
    want = [Fraction(v) for v in case["M_after"]]
    # every intermediate is an exact binary fraction: bit-exact
    assert [Fraction(float(v)) for v in M] == want
    assert r["capped_pairs"] == case["capped_pairs"]
    # a cap leaves its bin exactly empty, and those are the bins marked
    emptied = [case["capped_pairs"] > 0 and w == 0 for w in want]
    assert r["limited_bins"][0, 0].tolist() == emptied


def test_only_entries_with_i_le_j_are_read():
    # pair (i, j), i <= j, takes entry [i][j]; a lower triangle that holds
    # something else changes nothing
    case = _cases()[-1]
    B = case["nbins"]
    t = np.full((1, 1, B, B), case["K"])
    t[0, 0][np.tril_indices(B, -1)] = 7.0
    om = oracle.OracleModel(B, 1, t, np.array([1000.0]),
                            np.zeros((1, 1), np.int32), x1_g=1.0, order=1)
    N = np.array([[case["N"]]], dtype=np.float64)
    om.run(N, np.array([1000.0]), case["dt"], 1)
    M = N[0, 0] * om.grid()
    assert [Fraction(float(v)) for v in M] == \
        [Fraction(v) for v in case["M_after"]]


def test_worked_example_differs_from_simultaneous():
    case = _cases()[0]
    om = unit_grid_model(2, case["K"], order=0)
    N = np.array([[case["N"]]], dtype=np.float64)
    om.run(N, np.array([1000.0]), case["dt"], 1)
    assert list(N[0, 0] * om.grid()) == [0.5, 2.5]


def test_sequential_needs_one_species():
    w = wl.config3(npoints=4)
    with pytest.raises(ValueError):
        model_of(w, 1).grid()


def _thunderstorm_sample(n):
    w = wl.config2(nx=8, ny=8, nz=50)
    return w, w.subset(wl.sample_active(w, n))


def test_one_step_agrees_with_simultaneous_to_second_order():
    # each pair's first-order amount is the same in both forms; the forms
    # differ only through pairs acting on each other's results, O(dt^2)
    w, sub = _thunderstorm_sample(8)
    x = model_of(w, 0).grid()
    diffs = []
    for h in (8.0, 4.0, 2.0, 1.0):
        Na, Nb = sub.N.copy(), sub.N.copy()
        model_of(w, 0).run(Na, sub.p, h, 1)
        model_of(w, 1).run(Nb, sub.p, h, 1)
        change = np.abs((Na - sub.N) * x).sum()
        d = np.abs((Na - Nb) * x).sum()
        assert d < 0.25 * change
        diffs.append(d)
    ratios = [diffs[k] / diffs[k + 1] for k in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), ratios


def test_runs_converge_to_simultaneous_with_dt():
    w, sub = _thunderstorm_sample(8)
    x = model_of(w, 0).grid()
    diffs = []
    for dt in (4.0, 2.0, 1.0):
        n = int(round(40.0 / dt))
        Na, Nb = sub.N.copy(), sub.N.copy()
        model_of(w, 0).run(Na, sub.p, dt, n)
        model_of(w, 1).run(Nb, sub.p, dt, n)
        diffs.append(np.abs((Na - Nb) * x).sum())
    ratios = [diffs[k] / diffs[k + 1] for k in range(2)]
    assert all(1.8 < r < 2.2 for r in ratios), ratios


def _golovin(s):
    t_end = 1800.0
    w = wl.config1(npoints=1, s=s)
    om = model_of(w, 1)
    x = om.grid()
    N = w.N.copy()
    r = om.run(N, w.p, w.dt, w.nsteps)
    m = w.meta
    M = N[0, 0] * x
    Mex = cf.bin_masses(lambda xx: cf.golovin_n(xx, t_end, m["N0"],
                                                m["xbar"], m["b"]), x, s)
    l1 = np.abs(M - Mex).sum() / m["L"]
    num = N.sum() / cf.golovin_number(t_end, m["N0"], m["xbar"], m["b"])
    return l1, num, r["capped_pairs"], int(np.argmax(M)), int(np.argmax(Mex))


def test_golovin_refinement_ladder():
    res = {s: _golovin(s) for s in (1, 2, 4)}
    l1 = [res[s][0] for s in (1, 2, 4)]
    assert l1[0] / l1[1] >= 2.5 and l1[1] / l1[2] >= 2.5
    assert l1[0] < 0.55
    assert abs(res[1][1] - 1) < 0.16
    assert abs(res[2][1] - 1) < 0.05
    assert abs(res[4][1] - 1) < 0.015
    assert abs(res[1][3] - res[1][4]) <= 2
    assert all(res[s][2] == 0 for s in (1, 2, 4))


@pytest.mark.parametrize("dt", [2.0, 4000.0])
def test_laws(dt):
    w, sub = _thunderstorm_sample(16)
    om = model_of(w, 1)
    x = om.grid()
    N = sub.N.copy()
    prev = N.sum(axis=(1, 2))
    capped = 0
    for _ in range(5):
        r = om.run(N, sub.p, dt, 1)
        capped += r["capped_pairs"]
        assert np.all(N >= 0.0)
        tot = N.sum(axis=(1, 2))
        assert np.all(tot <= prev * (1 + 1e-14))
        prev = tot
    assert compare.drift(N, sub.N, x) <= 1e-13
    if dt > 1000.0:
        assert capped > 0      # the cap is what keeps this step positive
    else:
        assert capped == 0


@pytest.mark.parametrize("kernel", ["gravitational", "golovin"])
def test_well_conditioned_where_caps_fire(kernel):
    # a capped bin is left exactly empty; rounding residues of either sign
    # would be scaled by 2^(j-i) in later pairs, and one ulp of input
    # noise then moved the result by 1.2% at this time step (the Golovin
    # kernel also caps self pairs, which the gravitational one never does)
    w, sub = _thunderstorm_sample(96)
    if kernel == "golovin":
        w.tables = wl.golovin_tables(w.nbins)
        w.p_levels = np.array([1000.0])
    x = model_of(w, 1).grid()
    noise = np.random.default_rng(0).standard_normal(sub.N.shape)
    N1 = sub.N * (1.0 + 2e-16 * noise)
    outs, res = [], []
    for N in (sub.N.copy(), N1):
        res.append(model_of(w, 1).run(N, sub.p, 4000.0, 3))
        outs.append(N)
    assert res[0]["capped_pairs"] > 0
    # the wider floor only on the bins a cap emptied in the reference run
    floor = np.where(res[0]["limited_bins"], 1e-3, 1e-9)
    assert compare.rel_bin(outs[1], outs[0], x, floor=floor) < 1e-11


def test_determinism_and_threads():
    w, sub = _thunderstorm_sample(32)
    om = model_of(w, 1)
    outs = []
    for nt in (1, 3, 0):
        N = sub.N.copy()
        om.run(N, sub.p, w.dt, 10, nthreads=nt)
        outs.append(N)
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
