"""Analytic solutions of the stochastic collection equation.

TEST INFRASTRUCTURE ONLY (part of the oracle package).  These are the
textbook solutions used to pin the FP64 oracle, not part of the GPU path.

* Golovin (1963) / Scott (1968): sum kernel K(x, y) = b (x + y) with an
  exponential initial spectrum n0(x) = (N0 / xbar) exp(-x / xbar):
      n(x, t) = N0 (1 - T) / (x sqrt(T)) exp(-(1 + T) x / xbar)
                * I1(2 x sqrt(T) / xbar),            T = 1 - exp(-b L t),
  with L = N0 xbar the mass content.  Moments: N(t) = N0 exp(-b L t) and
  M2(t) = M2(0) exp(2 b L t).
* Constant kernel K = C, same initial spectrum:
      n(x, t) = 4 N0 / (xbar (2 + T)^2) exp(-2 x / (xbar (2 + T))),
  T = C N0 t;  N(t) = 2 N0 / (2 + T);  M2(t) = N0 xbar^2 (2 + T), since
  dM2/dt = C M1^2 with M1 = N0 xbar and M2(0) = 2 N0 xbar^2.

Bin discretisation on a logarithmic grid x_k = x_1 2^(k/s): the mass in bin k
is approximated by x_k^2 n(x_k) ln(2^(1/s)).
"""

from __future__ import annotations

import numpy as np
from scipy.special import ive


def golovin_n(x, t, N0, xbar, b):
    """Number density n(x, t) per unit mass for the Golovin kernel."""
    x = np.asarray(x, dtype=np.float64)
    L = N0 * xbar
    if t == 0:
        return N0 / xbar * np.exp(-x / xbar)
    T = -np.expm1(-b * L * t)
    z = 2.0 * x * np.sqrt(T) / xbar
    # I1(z) = ive(1, z) e^z keeps the product finite for large z
    return N0 * (1.0 - T) / (x * np.sqrt(T)) * np.exp(
        -(1.0 + T) * x / xbar + z) * ive(1, z)


def golovin_number(t, N0, xbar, b):
    return N0 * np.exp(-b * N0 * xbar * t)


def golovin_m2(t, N0, xbar, b):
    """Second mass moment: M2(0) = 2 N0 xbar^2 for the exponential start."""
    return 2.0 * N0 * xbar ** 2 * np.exp(2.0 * b * N0 * xbar * t)


def constant_n(x, t, N0, xbar, C):
    x = np.asarray(x, dtype=np.float64)
    T = C * N0 * t
    return 4.0 * N0 / (xbar * (2.0 + T) ** 2) * np.exp(
        -2.0 * x / (xbar * (2.0 + T)))


def constant_number(t, N0, C):
    return 2.0 * N0 / (2.0 + C * N0 * t)


def constant_m2(t, N0, xbar, C):
    """Second moment of the constant-kernel solution: N0 xbar^2 (2 + T)."""
    return N0 * xbar ** 2 * (2.0 + C * N0 * t)


def bin_masses(n_of_x, x, s):
    """Mass per bin on a grid with ratio 2^(1/s): x_k^2 n(x_k) ln 2 / s."""
    x = np.asarray(x, dtype=np.float64)
    return x * x * n_of_x(x) * (np.log(2.0) / s)
