"""Helpers shared by the GPU parity tests: oracle runs and the comparison
against the oracle at the stated tolerances.

Bar (per-bin mass error relative to max(|M_ref|, floor * M_tot), reading R15
of the collision step's open points):
  FP64 path 1e-12, FP32C path 1e-5, relative per-point mass drift 1e-10.
floor is 1e-9 for every bin, except for the bins the oracle's positivity
limiter scaled (sigma < 1 at some step of the call, reading R9) or, in the
sequential form, the bins a cap emptied: those get LIMITED_FLOOR.  The
limiter empties such a bin by the cancellation M - (M / D) D, so what is
left there (and whatever later steps grow from it) is rounding noise of
order u M_tot in either implementation; those bins, and only those, are
judged on that absolute scale, |dM| <= tol * 1e-3 * M_tot (1e-15 M_tot, a
few ulp of the point total, on the FP64 path).  Every other bin of a
limited point keeps the 1e-9 floor.

FP32C points whose own problem is ill-conditioned at FP32 precision
(reading R17): the activity threshold (R8) makes the step discontinuous in
the state, so a tail bin that crosses theta M_tot one step earlier or later
ends up different by far more than the rounding that decided it.  A point
over the FP32C tolerance counts as ill-conditioned only if the oracle
alone, run on the point's input perturbed by half an FP32 ulp (3e-8
relative, three seeded draws), moves by more than the tolerance.  A test
fails on any such point unless it passes an explicit allowance
(allow_ill_conditioned), and the count is always printed and part of the
assertion message.
"""

import numpy as np

import oracle
from oracle import compare

TOL = {0: 1e-12, 1: 1e-5}
DRIFT = 1e-10
FLOOR = 1e-9
LIMITED_FLOOR = 1e-3


class Limited:
    """What the oracle's limiter did in a run: per point, the steps at which
    it fired (sequential form: the capped pairs), and per bin whether it
    scaled (sequential form: emptied) that bin at some step."""

    def __init__(self, per_point, bins):
        self.per_point = np.asarray(per_point)
        self.bins = np.asarray(bins, dtype=bool)

    def sum(self):
        return int(self.per_point.sum())

    def points(self):
        """[P] bool: points at which the limiter acted."""
        return self.per_point > 0

    def __getitem__(self, idx):
        return Limited(self.per_point[idx], self.bins[idx])

    def repeat(self, n):
        """The same record for n copies of each point."""
        return Limited(np.repeat(self.per_point, n, axis=0),
                       np.repeat(self.bins, n, axis=0))

    def floor(self):
        """Per-bin rel_bin floors: LIMITED_FLOOR on the limited bins."""
        return np.where(self.bins, LIMITED_FLOOR, FLOOR)


def expected_kernel(w, precision, force_wave=False):
    """Kernel family a handle of workload w runs (fsbm_coal_stats.kernel):
    0 one point per lane (one species, doubling grid, B in 3/8/16/33/40),
    3 one point per lane for two to four species (FP32C, doubling grid, 33
    bins, pressure brackets x species sets within 64 buckets), else 1 (one
    point per wave)."""
    nbr = max(len(w.p_levels) - 1, 1)
    if force_wave:
        return 1
    if w.nspecies == 1 and w.s == 1 and w.nbins in (3, 8, 16, 33, 40):
        return 0
    if (precision == 1 and 2 <= w.nspecies <= 4 and w.s == 1 and
            w.nbins == 33 and nbr * (1 << w.nspecies) <= 64):
        return 3
    return 1


def model_of(w, order=0):
    return oracle.OracleModel(w.nbins, w.nspecies, w.tables, w.p_levels,
                              w.product, x1_g=w.x1_g, s=w.s, theta=w.theta,
                              order=order)


def run_oracle(w, N=None, p=None, dt=None, nsteps=None, order=0):
    """Oracle result, bin masses and the limiter record (Limited)."""
    om = model_of(w, order)
    Nr = np.array(w.N if N is None else N, dtype=np.float64, copy=True)
    res = om.run(Nr, w.p if p is None else p, w.dt if dt is None else dt,
                 w.nsteps if nsteps is None else nsteps)
    per_point = (res["capped_per_point"] if order == 1 else
                 res["limiter_per_point"])
    return Nr, om.grid(), Limited(per_point, res["limited_bins"])


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
          dt=None, nsteps=None, order=0, allow_ill_conditioned=0):
    """limited: the oracle run's Limited record (or None: no bin limited).
    w (the workload of got/ref, FP32C only): points over the tolerance are
    tested for ill-conditioning; at most allow_ill_conditioned of them may
    be excused."""
    P = ref.shape[0]
    if limited is None:
        limited = Limited(np.zeros(P, np.int32), np.zeros(ref.shape, bool))
    floor = limited.floor()
    n_over = n_ill = 0
    if precision == 1 and w is not None:
        pe = compare.per_point_rel_bin(got, ref, x, floor)
        over = np.nonzero(pe > TOL[1])[0]
        n_over = len(over)
        if n_over:
            ill = ill_conditioned(w, over, ref, floor, dt, nsteps, order)
            n_ill = int(ill.sum())
            print("%s: %d points over %.0e, %d of them ill-conditioned at "
                  "FP32 precision (errors %s)" % (
                      label, n_over, TOL[1], n_ill,
                      ["%.2e" % pe[q] for q in over]), flush=True)
            assert n_ill <= allow_ill_conditioned, (
                "%s: %d points excused as ill-conditioned at FP32 precision, "
                "%d allowed" % (label, n_ill, allow_ill_conditioned))
            keep = np.ones(P, dtype=bool)
            keep[over[ill]] = False
            got, ref, start, floor = got[keep], ref[keep], start[keep], \
                floor[keep]
            limited = limited[keep]
    err, worst = compare.rel_bin(got, ref, x, floor=floor, report=True)
    drift = compare.drift(got, start, x)
    nlim = int(limited.points().sum())
    if worst is not None:
        worst["limiter_steps"] = int(limited.per_point[worst["point"]])
        worst["limited_bin"] = bool(
            limited.bins[worst["point"], worst["species"], worst["bin"]])
    # the error of the limited points' other bins, on the 1e-9 floor alone
    err_lim = 0.0
    lp = limited.points()
    if lp.any():
        err_lim = compare.rel_bin(got[lp], ref[lp], x,
                                  floor=np.where(limited.bins[lp], np.inf,
                                                 FLOOR))
    print("%s precision=%d rel_bin=%.3e drift=%.3e limited_points=%d "
          "limited_bins=%d rel_bin_limited_points_other_bins=%.3e "
          "over_tol=%d ill_conditioned=%d worst=%s" % (
              label, precision, err, drift, nlim, int(limited.bins.sum()),
              err_lim, n_over, n_ill, worst), flush=True)
    assert np.all(got >= 0.0)
    assert err <= TOL[precision], (err, worst, "ill-conditioned excused: %d"
                                   % n_ill)
    assert drift <= DRIFT, drift
