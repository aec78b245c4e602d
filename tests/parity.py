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

FP32C points whose own problem is ill-conditioned at FP32 precision
(reading R17): the activity threshold (R8) makes the step discontinuous in
the state, so a tail bin that crosses theta M_tot one step earlier or later
ends up different by far more than the rounding that decided it.  A point
over the FP32C tolerance counts as ill-conditioned only if the oracle
alone, run on the point's input perturbed by half an FP32 ulp (3e-8
relative, three seeded draws), moves by more than the tolerance; such
points are reported and counted, every other point must meet the bar.
"""

import numpy as np

import oracle
from oracle import compare

TOL = {0: 1e-12, 1: 1e-5}
DRIFT = 1e-10
FLOOR = 1e-9
LIMITED_FLOOR = 1e-3


def model_of(w, order=0):
    return oracle.OracleModel(w.nbins, w.nspecies, w.tables, w.p_levels,
                              w.product, x1_g=w.x1_g, s=w.s, theta=w.theta,
                              order=order)


def run_oracle(w, N=None, p=None, dt=None, nsteps=None, order=0):
    """Oracle result, bin masses and per-point limiter step counts (order 1,
    the sequential form: per-point counts of capped pairs, which empty a
    bin by the same kind of cancellation)."""
    om = model_of(w, order)
    Nr = np.array(w.N if N is None else N, dtype=np.float64, copy=True)
    res = om.run(Nr, w.p if p is None else p, w.dt if dt is None else dt,
                 w.nsteps if nsteps is None else nsteps)
    lim = res["capped_per_point"] if order == 1 else res["limiter_per_point"]
    return Nr, om.grid(), lim


def ill_conditioned(w, idx, ref, floor, dt=None, nsteps=None, order=0):
    """Per point of idx (indices into w's points): True if the oracle's own
    result moves by more than the FP32C tolerance under input noise of half
    an FP32 ulp (see the module docstring)."""
    sub = w.subset(idx)
    om = model_of(w, order)
    return compare.unstable_points(
        om, sub.N, sub.p, w.dt if dt is None else dt,
        w.nsteps if nsteps is None else nsteps, ref[idx], om.grid(),
        floor[idx], TOL[1])


def check(got, ref, start, x, precision, label="", limited=None, w=None,
          dt=None, nsteps=None, order=0):
    """limited: per-point limiter step counts of the oracle run (or None).
    w (the workload of got/ref, FP32C only): points over the tolerance are
    tested for ill-conditioning and excused only if the oracle's own result
    is unstable at FP32 precision."""
    P = ref.shape[0]
    floor = np.full(P, FLOOR)
    if limited is not None:
        floor[np.asarray(limited) > 0] = LIMITED_FLOOR
    if precision == 1 and w is not None:
        pe = compare.per_point_rel_bin(got, ref, x, floor)
        over = np.nonzero(pe > TOL[1])[0]
        if len(over):
            ill = ill_conditioned(w, over, ref, floor, dt, nsteps, order)
            print("%s: %d points over %.0e, %d of them ill-conditioned at "
                  "FP32 precision (errors %s)" % (
                      label, len(over), TOL[1], int(ill.sum()),
                      ["%.2e" % pe[q] for q in over]), flush=True)
            keep = np.ones(P, dtype=bool)
            keep[over[ill]] = False
            got, ref, start, floor = got[keep], ref[keep], start[keep], \
                floor[keep]
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
