"""Pins of the condensation/evaporation oracle (readings R22-R25 in
oracle/fsbm_oracle_cond.c: the r dr/dt = G s growth law at a prescribed
supersaturation, the number- and mass-keeping two-moment remapping onto the
fixed grid, complete evaporation below the grid, the last bin holding what
grows past it), against what the growth law and the remapping fix:

* s = 0 is the identity, bit for bit;
* a drop population whose growth lands exactly on a grid point moves there
  whole (the growth for a doubling of mass is (2^(2/3) - 1) r^2);
* number is kept away from the grid's ends, and N >= 0; one step moves
  each bin's mass to exactly what the growth law gives its drops;
* a monodisperse population converges, as the grid is refined, to the
  exact r^2 law (liquid mass N vol (r0^2 + 2 G s t)^(3/2)): a refinement
  ladder;
* evaporation of everything returns the whole liquid mass as vapour;
  growth past the last bin keeps every drop in it.
A plausible slip (r instead of r^2 growth, a remap weight on the wrong
bin, a lost evaporation count, a search off by one) fails one of them.
"""

import numpy as np
import pytest

import oracle

X1 = 3.3510321638291124e-11   # 2 um water drop (g)
RHO = 1.0
VOL = 4.0 * np.pi * RHO / 3.0


def grid(B, s=1):
    k = np.arange(B)
    return np.ldexp(X1 * 2.0 ** ((k % s) / s), k // s)


def cond(N, ssat, G, dt, nsteps, s=1):
    N = np.array(N, dtype=np.float64, copy=True)
    ev = oracle.condense(N, np.broadcast_to(np.asarray(ssat, float),
                                            (N.shape[0],)).copy(),
                         np.broadcast_to(np.asarray(G, float),
                                         (N.shape[0],)).copy(),
                         dt, nsteps, s=s, x1_g=X1, rho=RHO)
    return N, ev


def test_zero_supersaturation_is_the_identity():
    rng = np.random.default_rng(1)
    N0 = rng.uniform(0.0, 5.0, (7, 33))
    N, ev = cond(N0, 0.0, 2e-6, 2.0, 10)
    assert np.array_equal(N, N0)
    assert np.all(ev == 0.0)


@pytest.mark.parametrize("k", [0, 5, 20])
def test_growth_to_a_grid_point_moves_the_bin_whole(k):
    B = 33
    x = grid(B)
    r2 = np.cbrt(x[k] / VOL) ** 2
    G, dt = 1e-6, 2.0
    ssat = (2.0 ** (2.0 / 3.0) - 1.0) * r2 / (2.0 * G * dt)
    N0 = np.zeros((1, B))
    N0[0, k] = 3.0
    N, ev = cond(N0, ssat, G, dt, 1)
    assert abs(N[0, k + 1] - 3.0) <= 1e-12 * 3.0
    assert np.all(N[0, :k + 1] <= 1e-12 * 3.0)
    assert np.all(N[0, k + 2:] <= 1e-12 * 3.0)
    assert ev[0] == 0.0


def test_number_kept_and_positive():
    rng = np.random.default_rng(2)
    B = 33
    N0 = np.zeros((50, B))
    N0[:, 8:21] = rng.uniform(0.0, 10.0, (50, 13))
    ssat = rng.uniform(-0.002, 0.01, 50)
    N, ev = cond(N0, ssat, 1.5e-6, 2.0, 20)
    assert np.all(N >= 0.0)
    # r^2 of bin 8 (1.6e-6 cm^2) is far above the 2.4e-7 cm^2 that 40 s of
    # evaporation at these rates removes: only the remapping's spread
    # (a fraction phi per step and bin) carries a trace below the grid
    x = grid(B)
    assert np.all(ev <= 1e-9 * (N0 @ x))
    lost = ev / x[0]   # at most this many drops left
    assert np.all(N.sum(axis=1) <= N0.sum(axis=1) * (1 + 1e-13))
    np.testing.assert_allclose(N.sum(axis=1), N0.sum(axis=1), rtol=1e-13,
                               atol=float(lost.max()))
    # the liquid mass changes by the growth of each drop (away from the
    # grid's top, which holds 1e-40 of the number here)
    gain = (N @ x) - (N0 @ x)
    assert np.all(np.sign(gain[ssat > 1e-4]) > 0)
    assert np.all(np.sign(gain[ssat < -1e-4]) < 0)


def test_one_step_moves_each_bin_mass_exactly():
    """Away from the grid's ends the remapping keeps number and mass of
    every source bin: after one step the liquid mass is sum N_k x'_k with
    x'_k = (4 pi / 3) (r_k^2 + 2 G s dt)^(3/2) from the growth law, and the
    number is unchanged, both to rounding."""
    rng = np.random.default_rng(6)
    for s in (1, 2, 4):
        B = 33 * s
        x = grid(B, s)
        r2 = np.cbrt(x / VOL) ** 2
        N0 = np.zeros((20, B))
        N0[:, 6 * s:20 * s] = rng.uniform(0.0, 3.0, (20, 14 * s))
        ssat = rng.uniform(-0.003, 0.01, 20)
        G, dt = 1.2e-6, 2.0
        N, ev = cond(N0, ssat, G, dt, 1, s=s)
        xnew = VOL * (r2[None, :] + 2.0 * G * ssat[:, None] * dt) ** 1.5
        assert np.all(ev == 0.0)
        np.testing.assert_allclose(N @ x, (N0 * xnew).sum(axis=1),
                                   rtol=1e-13)
        np.testing.assert_allclose(N.sum(axis=1), N0.sum(axis=1),
                                   rtol=1e-14)


def test_refinement_ladder_against_the_r2_law():
    """A monodisperse population (radius 10 um) at s = 0.5 %, G = 1e-6
    cm^2/s, 100 steps of 2 s: the liquid mass approaches the exact
    N vol (r0^2 + 2 G s t)^(3/2) as the bins per mass doubling go
    1, 2, 4, 8 (the remapping's numerical spread shrinks)."""
    G, ssat, dt, n = 1e-6, 0.005, 2.0, 100
    r0 = 10e-4
    exact = VOL * (r0 ** 2 + 2.0 * G * ssat * dt * n) ** 1.5
    errs = []
    for s in (1, 2, 4, 8):
        B = 33 * s
        x = grid(B, s)
        k0 = int(np.argmin(np.abs(x - VOL * r0 ** 3)))
        N0 = np.zeros((1, B))
        N0[0, k0] = 1.0
        x0 = x[k0]
        N, ev = cond(N0, ssat, G, dt, n, s=s)
        r0s = np.cbrt(x0 / VOL)
        ex = VOL * (r0s ** 2 + 2.0 * G * ssat * dt * n) ** 1.5
        errs.append(abs(float(N[0] @ x) - ex) / ex)
        assert abs(N.sum() - 1.0) < 1e-13
    assert exact > 0.0
    # first order in the bin width: 3.7e-2, 1.8e-2, 8.4e-3, 3.7e-3
    for a, b in zip(errs, errs[1:]):
        assert b < a / 1.8, errs
    assert errs[-1] < 0.005, errs


def test_evaporation_and_the_grid_ends():
    rng = np.random.default_rng(4)
    B = 33
    x = grid(B)
    N0 = rng.uniform(0.0, 2.0, (3, B))
    liquid = N0 @ x
    # everything evaporates: r^2 falls below 0 for every bin in one step
    r2max = np.cbrt(x[-1] / VOL) ** 2
    N, ev = cond(N0, -1.0, r2max, 1.0, 1)
    assert np.all(N == 0.0)
    np.testing.assert_allclose(ev, liquid, rtol=1e-14)
    # everything grows past the last bin and stays in it
    N, ev = cond(N0, 1.0, 10.0 * r2max, 1.0, 1)
    np.testing.assert_allclose(N[:, -1], N0.sum(axis=1), rtol=1e-14)
    assert np.all(N[:, :-1] == 0.0) and np.all(ev == 0.0)


def test_bad_input_refused():
    N = np.zeros((1, 33))
    with pytest.raises(ValueError):
        cond(N, 0.01, 1e-6, 0.0, 1)
    with pytest.raises(ValueError):
        oracle.condense(N, np.zeros(1), np.zeros(1), 1.0, 1, s=0)
