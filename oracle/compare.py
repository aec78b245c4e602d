"""Error metrics between a candidate state and the oracle's state.

TEST INFRASTRUCTURE ONLY (part of the oracle package).

rel_bin: max over points, species and bins of
    |M_cand - M_ref| / max(|M_ref|, 1e-9 * M_tot,ref)
so bins holding less than 1e-9 of their point's mass are judged on an
absolute scale.  drift: max over points of |sum M_end - sum M_0| / sum M_0.
"""

from __future__ import annotations

import numpy as np


def masses(N: np.ndarray, x: np.ndarray) -> np.ndarray:
    """[P][S][B] numbers -> masses."""
    return N * x[None, None, :]


def _floor_array(floor, shape):
    """floor as [P][S][B]: a scalar, one value per point ([P]) or one per
    bin ([P][S][B])."""
    fl = np.asarray(floor, dtype=np.float64)
    if fl.ndim == 1:
        fl = fl[:, None, None]
    return np.broadcast_to(fl, shape)


def rel_bin(N_cand, N_ref, x, floor=1e-9, report=False):
    """floor: scalar, per-point [P] or per-bin [P][S][B] array (fraction of
    the point's total mass below which a bin is judged on absolute error).
    With report=True also returns the worst (point, species, bin) and its
    masses relative to the point total."""
    Mc = masses(np.asarray(N_cand, dtype=np.float64), x)
    Mr = masses(np.asarray(N_ref, dtype=np.float64), x)
    P = Mr.shape[0]
    tot = Mr.reshape(P, -1).sum(axis=1)
    fl = _floor_array(floor, Mr.shape)
    den = np.maximum(np.abs(Mr), fl * tot[:, None, None])
    err = np.abs(Mc - Mr)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(den > 0, err / np.where(den > 0, den, 1.0),
                     np.where(err > 0, np.inf, 0.0))
    if report:
        if not r.size:
            return 0.0, None
        w = np.unravel_index(int(np.argmax(r)), r.shape)
        t = tot[w[0]] if tot[w[0]] > 0 else 1.0
        return float(r.max()), {"point": int(w[0]), "species": int(w[1]),
                                "bin": int(w[2]), "ref_frac": Mr[w] / t,
                                "cand_frac": Mc[w] / t}
    return float(r.max()) if r.size else 0.0


def drift(N_end, N_start, x):
    P = N_start.shape[0]
    m0 = masses(N_start, x).reshape(P, -1).sum(axis=1)
    m1 = masses(N_end, x).reshape(P, -1).sum(axis=1)
    ok = m0 > 0
    if not ok.any():
        return 0.0
    return float(np.max(np.abs(m1[ok] - m0[ok]) / m0[ok]))


def l1_point(N_cand, N_ref, x):
    Mc = masses(N_cand, x)
    Mr = masses(N_ref, x)
    P = Mr.shape[0]
    tot = Mr.reshape(P, -1).sum(axis=1)
    d = np.abs(Mc - Mr).reshape(P, -1).sum(axis=1)
    ok = tot > 0
    return float(np.max(d[ok] / tot[ok])) if ok.any() else 0.0


def per_point_rel_bin(N_cand, N_ref, x, floor=1e-9):
    """rel_bin of each point separately ([P]); floor as in rel_bin."""
    N_ref = np.asarray(N_ref, dtype=np.float64)
    fl = _floor_array(floor, N_ref.shape)
    return np.array([rel_bin(N_cand[q:q + 1], N_ref[q:q + 1], x,
                             floor=fl[q:q + 1]) for q in range(N_ref.shape[0])])


# Conditioning at FP32 precision: the activity threshold makes the step
# discontinuous in the state, so where a bin of a point crosses it near a
# step boundary the point's result jumps under rounding-sized changes of
# the input.  Such a point is recognised by the oracle alone: its result
# moves by more than tol under input noise of half an FP32 ulp.
COND_AMP = 3e-8
COND_SEEDS = (0, 1, 2)


def unstable_points(model, N, p, dt, nsteps, ref, x, floor, tol,
                    amp=COND_AMP, seeds=COND_SEEDS):
    """model: an oracle.OracleModel; N, p: the points' inputs; ref: the
    oracle's result for them; floor: rel_bin floors (per point or per bin).
    True where some seeded perturbation N (1 + amp z) moves the oracle's
    result by more than tol (rel_bin against ref)."""
    N = np.asarray(N, dtype=np.float64)
    P = N.shape[0]
    fl = _floor_array(floor, N.shape)
    out = np.zeros(P, dtype=bool)
    for seed in seeds:
        z = np.random.default_rng(seed).standard_normal(N.shape)
        Np = np.ascontiguousarray(N * (1.0 + amp * z))
        model.run(Np, p, dt, nsteps)
        out |= per_point_rel_bin(Np, ref, x, fl) > tol
    return out
