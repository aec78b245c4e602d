"""Pins of the sedimentation oracle (the vertical term of eq. (1), readings
R18-R21 in oracle/fsbm_oracle_sed.c), by properties that the first-order
upwind flux form must have and that a plausible slip (a flux taken from the
wrong level, a missing sub-step, a wrong thickness, a dropped or doubled
outflow) breaks:

* conservation: column content plus precipitation is constant (rounding);
* Courant number 1 on a uniform grid: a profile moves down one level per
  step, exactly; with per-level factors that make every level's Courant
  number 1 (or 1/2) the content moves (or spreads binomially) the same
  way on an uneven grid;
* uniform Courant number C < 1: a single-level pulse spreads as the
  binomial distribution of n trials with probability C (the scheme's own
  closed form, N_l' = (1 - C) N_l + C N_{l+1});
* the first moment moves down at exactly v while nothing reaches the
  ground; each bin falls at its own speed, independently;
* sub-steps: a step with Courant number 2.5 equals three steps of a third
  of it; positivity for any Courant number;
* layouts: level-major and column-major grids give the same result.
"""

import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def _sed(N, dz, v, dt, nsteps, vfac=None, col_stride=None, lev_stride=None):
    N = np.array(N, dtype=np.float64, copy=True)
    pr = oracle.sediment(N, dz, v, dt, nsteps, vfac=vfac,
                         col_stride=col_stride, lev_stride=lev_stride)
    return N, pr


def test_courant_one_shifts_exactly():
    nlev, S, B = 12, 1, 3
    dz = np.full(nlev, 250.0)
    v = np.array([[100.0, 50.0, 25.0]])          # cm/s
    dt = 2.5                                    # C = 1 for bin 0
    N = np.zeros((1, nlev, S, B))
    N[0, :, 0, 0] = np.arange(1.0, nlev + 1.0)
    out, pr = _sed(N, dz, v, dt, 3)
    # bin 0: down three levels, the lowest three have left
    np.testing.assert_array_equal(out[0, :nlev - 3, 0, 0],
                                  N[0, 3:, 0, 0])
    np.testing.assert_array_equal(out[0, nlev - 3:, 0, 0], 0.0)
    assert pr[0, 0, 0] == (1.0 + 2.0 + 3.0) * 250.0


@pytest.mark.parametrize("C", [0.25, 0.6, 0.9])
def test_pulse_spreads_binomially(C):
    nlev, L0, n = 40, 30, 12
    dz = np.full(nlev, 100.0)
    v = np.array([[C * 100.0 / 2.0]])
    N = np.zeros((1, nlev, 1, 1))
    N[0, L0, 0, 0] = 7.0
    out, pr = _sed(N, dz, v, 2.0, n)
    for k in range(n + 1):
        exact = 7.0 * math.comb(n, k) * C ** k * (1 - C) ** (n - k)
        assert abs(out[0, L0 - k, 0, 0] - exact) <= 1e-13 * 7.0, k
    assert np.count_nonzero(out) == n + 1
    assert pr[0, 0, 0] == 0.0


def test_level_and_column_factors():
    """Fall-speed factors per column and level: with v_l dt = dz_l at every
    level (column 0) the content N_l dz_l moves down one level per step;
    with half of it (column 1) the content spreads binomially with C = 1/2,
    whatever the layer thicknesses."""
    rng = np.random.default_rng(4)
    nlev, n, L0 = 24, 6, 20
    # thicknesses of 128 to 1024 cm: every factor and Courant number exact
    dz = 2.0 ** rng.integers(7, 11, nlev)
    v = np.array([[64.0]])
    vfac = np.stack([dz / 128.0, dz / 256.0])
    N = np.zeros((2, nlev, 1, 1))
    N[:, L0, 0, 0] = 3.0 / dz[L0]
    out, pr = _sed(N, dz, v, 2.0, n, vfac=vfac)
    content = out[:, :, 0, 0] * dz[None, :]
    for k in range(nlev):
        c0 = 3.0 if k == L0 - n else 0.0
        assert abs(content[0, k] - c0) <= 1e-12 * 3.0, k
        kk = L0 - k
        c1 = (3.0 * math.comb(n, kk) * 0.5 ** n) if 0 <= kk <= n else 0.0
        assert abs(content[1, k] - c1) <= 1e-12 * 3.0, k


def test_conservation_and_positivity_random_columns():
    rng = np.random.default_rng(5)
    ncol, nlev, S, B = 9, 23, 2, 5
    dz = rng.uniform(80.0, 400.0, nlev)
    v = rng.uniform(0.0, 600.0, (S, B))          # up to C = 15 per step
    vfac = rng.uniform(1.0, 1.4, (ncol, nlev))
    N = rng.uniform(0.0, 10.0, (ncol, nlev, S, B))
    N[rng.random(N.shape) < 0.3] = 0.0
    out, pr = _sed(N, dz, v, 2.0, 17, vfac=vfac)
    assert np.all(out >= 0.0)
    before = np.einsum("clsb,l->csb", N, dz)
    after = np.einsum("clsb,l->csb", out, dz) + pr
    np.testing.assert_allclose(after, before, rtol=1e-13, atol=0.0)


def test_first_moment_moves_at_the_fall_speed():
    rng = np.random.default_rng(8)
    nlev = 200
    dz = np.full(nlev, 50.0)
    v = np.array([[7.0, 13.0, 0.0]])
    N = np.zeros((1, nlev, 1, 3))
    N[0, 150:170, 0, :] = rng.uniform(1.0, 2.0, (20, 3))
    out, pr = _sed(N, dz, v, 3.0, 40)             # 840 / 1560 cm down
    z = (np.arange(nlev) + 0.5) * 50.0
    for k, vk in enumerate(v[0]):
        m0 = np.sum(N[0, :, 0, k] * z) / np.sum(N[0, :, 0, k])
        m1 = np.sum(out[0, :, 0, k] * z) / np.sum(out[0, :, 0, k])
        assert abs((m0 - m1) - vk * 3.0 * 40) <= 1e-9 * m0, k
    # a bin that does not fall stays put, bit for bit
    np.testing.assert_array_equal(out[0, :, 0, 2], N[0, :, 0, 2])
    assert np.all(pr == 0.0)


def test_sub_steps_split_a_long_step():
    """C = 2.5 in one step is three sub-steps of C = 2.5 / 3."""
    rng = np.random.default_rng(3)
    nlev = 30
    dz = np.full(nlev, 100.0)
    N = rng.uniform(0.0, 5.0, (1, nlev, 1, 1))
    a, pa = _sed(N, dz, np.array([[125.0]]), 2.0, 1)
    b, pb = _sed(N, dz, np.array([[125.0]]), 2.0 / 3.0, 3)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(pa, pb)
    assert np.all(a >= 0.0)


def test_level_major_layout_equals_column_major():
    rng = np.random.default_rng(11)
    nx, ny, nz, S, B = 4, 3, 10, 1, 4
    dz = rng.uniform(100.0, 300.0, nz)
    v = rng.uniform(0.0, 200.0, (S, B))
    Ncol = rng.uniform(0.0, 3.0, (nx * ny, nz, S, B))
    a, pa = _sed(Ncol, dz, v, 2.0, 5)
    # [nz][ny*nx] order: column stride 1, level stride nx*ny
    Nlev = np.ascontiguousarray(np.transpose(Ncol, (1, 0, 2, 3)))
    b, pb = _sed(Nlev, dz, v, 2.0, 5, col_stride=1, lev_stride=nx * ny)
    np.testing.assert_array_equal(np.transpose(b, (1, 0, 2, 3)), a)
    np.testing.assert_array_equal(pa, pb)


def test_bad_input_refused():
    N = np.zeros((1, 3, 1, 1))
    with pytest.raises(ValueError):
        _sed(N, np.array([1.0, 0.0, 1.0]), np.array([[1.0]]), 1.0, 1)
    with pytest.raises(ValueError):
        _sed(N, np.ones(3), np.array([[-1.0]]), 1.0, 1)
    with pytest.raises(ValueError):
        _sed(N, np.ones(3), np.array([[1.0]]), 0.0, 1)
