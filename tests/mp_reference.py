"""Tiny-case cross-check of the collision step in 50-digit arithmetic.

A second, independent transcription of the step (mass from numbers, activity
threshold, per-point pressure interpolation, canonical pair loop with the
exponential-profile flux fraction, limiter, update), written in plain Python
over mpmath numbers for B <= 6.  It shares no code with the C oracle and is
used only to catch indexing and ordering slips in it on tiny inputs; the
physics pins are the closed forms, invariants and worked examples in
test_oracle_pins.py.
"""

from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50


def grid(B, s, x1):
    return [mp.ldexp(mp.mpf(x1) * mp.power(2, mp.mpf(k % s) / s), k // s)
            for k in range(B)]


def targets(x, B, s, x1):
    def gm(k):
        return mp.ldexp(mp.mpf(x1) * mp.power(2, mp.mpf(k % s) / s), k // s)

    kt = [[0] * B for _ in range(B)]
    ct = [[mp.mpf(0)] * B for _ in range(B)]
    for i in range(B):
        for j in range(B):
            sm = x[i] + x[j]
            k = 0
            while gm(k + 1) <= sm * (1 + mp.mpf("1e-12")):
                k += 1
            if k >= B:
                kt[i][j] = -1
                continue
            kt[i][j] = k
            if k <= B - 2:
                c = (sm - x[k]) / (x[k + 1] - x[k])
                ct[i][j] = min(max(c, mp.mpf(0)), mp.mpf(1))
    return kt, ct


def flux_fraction(c, x1):
    if c == 0:
        return mp.mpf(0)
    if x1 == 0:
        f = c
    else:
        f = mp.exp((mp.mpf("0.5") - c) * x1) * mp.expm1(c * x1) / x1
    return min(max(f, mp.mpf(0)), mp.mpf(1))


def kernel(tables, plev, S, a, b, i, j, p):
    ab = a * S - a * (a - 1) // 2 + (b - a)
    L = len(plev)
    if L == 1:
        return mp.mpf(tables[ab][0][i][j])
    p = min(max(mp.mpf(p), mp.mpf(plev[-1])), mp.mpf(plev[0]))
    l = 0
    while l < L - 2 and not (plev[l] >= p >= plev[l + 1]):
        l += 1
    w = (p - plev[l + 1]) / (mp.mpf(plev[l]) - plev[l + 1])
    k0 = mp.mpf(tables[ab][l][i][j])
    k1 = mp.mpf(tables[ab][l + 1][i][j])
    return k1 + (k0 - k1) * w


def step(N, p, dt, B, S, s, x1, tables, plev, product, theta=1e-30):
    """One step of one point.  N: list [S][B] of mpf (replaced)."""
    x = grid(B, s, x1)
    kt, ct = targets(x, B, s, x1)
    M = [[N[a][k] * x[k] for k in range(B)] for a in range(S)]
    Mtot = mp.fsum(M[a][k] for a in range(S) for k in range(B))
    if Mtot == 0:
        return N
    act = [[M[a][k] > 0 and M[a][k] >= theta * Mtot for k in range(B)]
           for a in range(S)]
    Mt = [[M[a][k] if act[a][k] else mp.mpf(0) for k in range(B)]
          for a in range(S)]
    floor = -60 * mp.log(10)

    pairs = []  # list of dict bin->amount (merged)
    for a in range(S):
        for b in range(a, S):
            for i in range(B):
                if not act[a][i]:
                    continue
                for j in range(i if a == b else 0, B):
                    if not act[b][j]:
                        continue
                    k = kt[i][j]
                    if k < 0:
                        continue
                    K = kernel(tables, plev, S, a, b, i, j, p)
                    C = dt * K * N[a][i] * N[b][j]
                    if a == b and i == j:
                        C = C / 2
                    if C == 0:
                        continue
                    A = C * x[i]
                    Bm = C * x[j]
                    Sm = A + Bm
                    P = product[a][b]
                    F = mp.mpf(0)
                    if k <= B - 2:
                        r = Mt[P][k + 1] / (Mt[P][k] + Sm)
                        x1v = mp.log(r) if r > 0 else floor
                        x1v = max(x1v, floor)
                        F = flux_fraction(ct[i][j], x1v) * Sm
                    d = {}
                    for key, v in (((a, i), -A), ((b, j), -Bm),
                                   ((P, k), Sm - F)):
                        d[key] = d.get(key, 0) + v
                    if k <= B - 2:
                        d[(P, k + 1)] = d.get((P, k + 1), 0) + F
                    pairs.append(d)
    D = {}
    for d in pairs:
        for key, v in d.items():
            if v < 0:
                D[key] = D.get(key, 0) - v
    sig = {key: (min(mp.mpf(1), M[key[0]][key[1]] / v) if v > 0 else 1)
           for key, v in D.items()}
    limited = any(v > M[key[0]][key[1]] for key, v in D.items())
    net = [[mp.mpf(0)] * B for _ in range(S)]
    for d in pairs:
        scale = mp.mpf(1)
        if limited:
            for key, v in d.items():
                if v < 0:
                    scale = min(scale, sig[key])
        for key, v in d.items():
            net[key[0]][key[1]] += v * scale
    out = [[mp.mpf(0)] * B for _ in range(S)]
    for a in range(S):
        for k in range(B):
            m = M[a][k] + net[a][k]
            if m < 0:
                m = mp.mpf(0)
            out[a][k] = m / x[k]
    return out
