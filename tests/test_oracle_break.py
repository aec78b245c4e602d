"""Pins of the spontaneous-breakup oracle (readings R26-R28 in
oracle/fsbm_oracle_break.c: a drop of bin l breaks at the rate P_l into
Q[l][k] fragments in each smaller bin k; over a step the share
1 - exp(-P dt) of a bin breaks and its fragments do not break again within
the step), against what the equation fixes:

* P = 0 is the identity, bit for bit;
* mass is kept to the fragment table's own balance, N >= 0, the number
  never falls;
* one bin breaking into two drops of the bin below it decays exactly as
  exp(-P t) (the loss term's closed form), and the fragments hold the
  rest;
* as dt -> 0 at fixed n dt the result converges, at first order, to the
  exact solution exp(T M) N_0 of the linear system;
* bad tables are refused.
A plausible slip (fragments transposed, the loss term dropped, P dt in
place of 1 - exp(-P dt), the fragment sum running the wrong way) fails one
of them.
"""

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2409_07232_amd import workloads as wl


def brk(N, rate, Q, dt, nsteps):
    N = np.array(N, dtype=np.float64, copy=True)
    oracle.breakup(N, rate, Q, dt, nsteps)
    return N


def test_zero_rates_are_the_identity():
    rng = np.random.default_rng(1)
    N0 = rng.uniform(0.0, 5.0, (6, 33))
    _, Q = wl.breakup_tables(33)
    N = brk(N0, np.zeros(33), Q, 2.0, 10)
    assert np.array_equal(N, N0)


@pytest.mark.parametrize("B,s", [(33, 1), (66, 2)])
def test_mass_kept_number_grows_positive(B, s):
    rng = np.random.default_rng(B)
    rate, Q = wl.breakup_tables(B, s)
    x = wl.bin_masses(B, s)
    N0 = rng.uniform(0.0, 1.0, (40, B)) * np.exp(-rng.uniform(0, 0.5, (40, 1))
                                                * np.arange(B))
    N = N0.copy()
    for _ in range(5):
        prev = N.copy()
        N = brk(N, rate, Q, 2.0, 3)
        assert np.all(N >= 0.0)
        assert np.all(N.sum(axis=1) >= prev.sum(axis=1) * (1 - 1e-15))
    np.testing.assert_allclose(N @ x, N0 @ x, rtol=1e-13)
    # the largest drops (P dt >> 1) are gone, the small ones gained
    assert np.all(N[:, -1] < 1e-12 * N0[:, -1])
    assert np.all(N[:, 0] > N0[:, 0])


def test_one_bin_into_two_exact_decay():
    """Bin 10 (P = 0.3 /s) breaks into two drops of bin 9 (half its mass on
    the doubling grid); nothing else breaks: N_10 = N0 exp(-P t),
    N_9 = 2 (N0 - N_10)."""
    B = 33
    rate = np.zeros(B)
    rate[10] = 0.3
    Q = np.zeros((B, B))
    Q[10, 9] = 2.0
    N0 = np.zeros((1, B))
    N0[0, 10] = 7.0
    for n in (1, 5, 40):
        N = brk(N0, rate, Q, 0.5, n)
        exact = 7.0 * np.exp(-0.3 * 0.5 * n)
        assert abs(N[0, 10] - exact) <= 1e-13 * 7.0
        assert abs(N[0, 9] - 2.0 * (7.0 - N[0, 10])) <= 1e-13 * 14.0
        assert np.count_nonzero(N) == 2


def test_dt_ladder_to_the_matrix_exponential():
    """Twelve bins, rates up to 0.5 /s, T = 4 s: the error against
    exp(T M) N_0 halves as dt halves (1.2e-1 at 8 steps, 7.7e-3 at
    128)."""
    B = 12
    x = wl.bin_masses(B)
    rate = np.linspace(0.0, 0.5, B)
    _, Q = wl.breakup_tables(B)
    M = np.zeros((B, B))
    for l in range(1, B):
        M[l, l] -= rate[l]
        M[:l, l] += rate[l] * Q[l, :l]
    N0 = np.exp(-0.3 * np.arange(B))[None, :]
    exact = scipy.linalg.expm(4.0 * M) @ N0[0]
    errs = []
    for n in (8, 16, 32, 64, 128):
        N = brk(N0, rate, Q, 4.0 / n, n)
        errs.append(np.abs(N[0] - exact).max() / exact.max())
    for a, b in zip(errs, errs[1:]):
        assert 1.8 < a / b < 2.2, errs
    assert errs[-1] < 0.01, errs
    # and mass is kept along the way
    np.testing.assert_allclose(N @ x, N0 @ x, rtol=1e-13)


def test_bad_tables_refused():
    rate, Q = wl.breakup_tables(8)
    N = np.zeros((1, 8))
    Qd = Q.copy()
    Qd[3, 3] = 1.0
    with pytest.raises(ValueError):
        brk(N, rate, Qd, 1.0, 1)
    Qu = Q.copy()
    Qu[2, 5] = 0.5
    with pytest.raises(ValueError):
        brk(N, rate, Qu, 1.0, 1)
    r = rate.copy()
    r[4] = -1.0
    with pytest.raises(ValueError):
        brk(N, r, Q, 1.0, 1)
    with pytest.raises(ValueError):
        brk(N, rate, Q, 0.0, 1)
