"""Helpers shared by the GPU parity tests: oracle runs and the comparison
against the oracle at the stated tolerances.

Bar (per-bin mass error relative to max(|M_ref|, floor * M_tot), reading R15
of the collision step's open points):
  FP64 path 1e-12, FP32C path 1e-5, relative per-point mass drift 1e-10.
floor is 1e-9 for ordinary points.  For a point whose oracle run applied the
positivity limiter (reading R9) the floor is LIMITED_FLOOR: the limiter
empties an over-demanded bin by the cancellation M - (M / D) D, so what is
left there (and whatever later steps grow from it) is rounding noise of
order u M_tot in either implementation; such bins are judged on that
absolute scale, i.e. |dM| <= tol * 1e-3 * M_tot (1e-15 M_tot, a few ulp of
the point total, on the FP64 path).
"""

import numpy as np

import oracle
from oracle import compare

TOL = {0: 1e-12, 1: 1e-5}
DRIFT = 1e-10
FLOOR = 1e-9
LIMITED_FLOOR = 1e-3


def model_of(w):
    return oracle.OracleModel(w.nbins, w.nspecies, w.tables, w.p_levels,
                              w.product, x1_g=w.x1_g, s=w.s, theta=w.theta)


def run_oracle(w, N=None, p=None, dt=None, nsteps=None):
    """Oracle result, bin masses and per-point limiter step counts."""
    om = model_of(w)
    Nr = np.array(w.N if N is None else N, dtype=np.float64, copy=True)
    res = om.run(Nr, w.p if p is None else p, w.dt if dt is None else dt,
                 w.nsteps if nsteps is None else nsteps)
    return Nr, om.grid(), res["limiter_per_point"]


def check(got, ref, start, x, precision, label="", limited=None):
    """limited: per-point limiter step counts of the oracle run (or None)."""
    P = ref.shape[0]
    floor = np.full(P, FLOOR)
    if limited is not None:
        floor[np.asarray(limited) > 0] = LIMITED_FLOOR
    err, worst = compare.rel_bin(got, ref, x, floor=floor, report=True)
    drift = compare.drift(got, start, x)
    nlim = 0 if limited is None else int((np.asarray(limited) > 0).sum())
    if worst is not None and limited is not None:
        worst["limiter_steps"] = int(np.asarray(limited)[worst["point"]])
    print("%s precision=%d rel_bin=%.3e drift=%.3e limited_points=%d "
          "worst=%s" % (label, precision, err, drift, nlim, worst),
          flush=True)
    assert np.all(got >= 0.0)
    assert err <= TOL[precision], (err, worst)
    assert drift <= DRIFT, drift
