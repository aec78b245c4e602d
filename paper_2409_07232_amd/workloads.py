"""Seeded synthetic inputs for the collision step.

This module only DECIDES INPUTS: bin grids used to lay out spectra and kernel
tables, collection-kernel tables at pressure levels, initial spectra, cloudy
masks and point pressures.  It holds none of the collision arithmetic and is
shared by the GPU tests and the oracle tests alike.

The paper benchmarks on the CONUS-12km WRF case (425 x 300 x 50 points,
dt = 5 s; Sec. IV) whose data and FSBM kernel files are not available here.
These generators stand in for them with the shapes of that workload: 33 mass
doubling bins per particle type (Sec. III), kernel tables at several pressure
levels interpolated per point (Sec. VI-A), and a minority of cloudy points
(Sec. VIII discusses that many cells hold no cloud).

Seeds: numpy PCG64(240907232 + config_id).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 240907232
RHO_WATER = 1.0                                   # g cm^-3
R1_CM = 2.0e-4                                    # 2 um smallest drop
X1_G = 4.0 / 3.0 * np.pi * R1_CM ** 3 * RHO_WATER  # 3.351e-11 g
P_LEVELS_3 = np.array([1000.0, 750.0, 500.0])

# Config-3 species: liquid drops, ice crystals, snow, graupel.
SPECIES_4 = ("liquid", "ice", "snow", "graupel")
BETA_4 = (0.8, 0.3, 0.4, 0.6)
RHO_4 = (1.0, 0.9, 0.1, 0.4)
# Initial spectra per species: gamma mean radius (cm) and the log-uniform
# range of the species content (g/m^3).  Ice species are fewer and larger
# than cloud drops, so per-bin collection rates stay below one per 2 s step
# at almost every point (the positivity limiter is the exception).
RBAR_4 = (10.0e-4, 100.0e-4, 300.0e-4, 500.0e-4)
CONTENT_4 = ((0.1, 3.0), (0.01, 0.3), (0.01, 0.5), (0.01, 1.0))
# product species of a collision, symmetric: riming keeps the collector's
# ice species (l+i->i, l+s->s, l+g->g), aggregation of crystals and snow
# gives snow (i+i->s, i+s->s, s+s->s), anything with graupel stays graupel.
PRODUCT_4 = np.array([[0, 1, 2, 3],
                      [1, 2, 2, 3],
                      [2, 2, 2, 3],
                      [3, 3, 3, 3]], dtype=np.int32)
# Config-4 species: liquid and graupel.
PRODUCT_2 = np.array([[0, 1], [1, 1]], dtype=np.int32)


@dataclass
class Workload:
    """One bin grid with its species set, tables and point states."""

    name: str
    nbins: int
    nspecies: int
    s: int
    tables: np.ndarray            # [S(S+1)/2][L][B][B] float64, cm^3/s
    p_levels: np.ndarray          # [L] hPa, strictly decreasing
    product: np.ndarray           # [S][S] int32
    N: np.ndarray                 # [P][S][B] float64, cm^-3 per bin
    p: np.ndarray                 # [P] float64, hPa
    dt: float
    nsteps: int
    x1_g: float = X1_G
    theta: float = 1e-30
    meta: dict = field(default_factory=dict)

    @property
    def npoints(self) -> int:
        return int(self.N.shape[0])

    def cloudy(self) -> np.ndarray:
        return np.any(self.N.reshape(self.npoints, -1) > 0.0, axis=1)

    def subset(self, idx) -> "Workload":
        """The same model on a subset of its points (copied)."""
        idx = np.asarray(idx)
        return Workload(self.name + "[subset]", self.nbins, self.nspecies,
                        self.s, self.tables, self.p_levels, self.product,
                        np.ascontiguousarray(self.N[idx]),
                        np.ascontiguousarray(self.p[idx]), self.dt,
                        self.nsteps, self.x1_g, self.theta, dict(self.meta))


def rng_for(config_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config_id))


def bin_masses(nbins: int, s: int = 1, x1: float = X1_G) -> np.ndarray:
    """x_k = x_1 2^(k/s), built with ldexp so that doubling is exact."""
    k = np.arange(nbins)
    return np.ldexp(x1 * np.power(2.0, (k % s) / s), k // s)


def radius_cm(x_g, rho):
    return np.cbrt(3.0 * np.asarray(x_g) / (4.0 * np.pi * rho))


def golovin_tables(nbins, s=1, b=1500.0, x1=X1_G, nlevels=1):
    """K_ij = b (x_i + x_j), identical at every level, one species."""
    x = bin_masses(nbins, s, x1)
    K = b * (x[:, None] + x[None, :])
    return np.ascontiguousarray(np.broadcast_to(K, (1, nlevels, nbins,
                                                    nbins)))


def constant_tables(nbins, C, nlevels=1):
    return np.full((1, nlevels, nbins, nbins), float(C))


def gravitational_tables(nbins, s, rho, beta, vcoef, p_levels,
                         x1=X1_G):
    """Hydrodynamic kernel K = pi (r_a + r_b)^2 |v_a - v_b| (efficiency 1)
    for every species pair a <= b, at each pressure level, with fall speeds
    v = vcoef_a r^beta_a (cm/s, r in cm) scaled by (1000 / p)^0.4."""
    S = len(rho)
    x = bin_masses(nbins, s, x1)
    r = [radius_cm(x, rho[a]) for a in range(S)]
    npairs = S * (S + 1) // 2
    L = len(p_levels)
    out = np.empty((npairs, L, nbins, nbins))
    q = 0
    for a in range(S):
        for b in range(a, S):
            for li, pl in enumerate(p_levels):
                scale = (1000.0 / pl) ** 0.4
                va = vcoef[a] * r[a] ** beta[a] * scale
                vb = vcoef[b] * r[b] ** beta[b] * scale
                out[q, li] = (np.pi * (r[a][:, None] + r[b][None, :]) ** 2 *
                              np.abs(va[:, None] - vb[None, :]))
            q += 1
    return out


def liquid_tables(nbins, s=1, p_levels=P_LEVELS_3):
    return gravitational_tables(nbins, s, (RHO_WATER,), (0.8,), (8.0e3,),
                                p_levels)


def multi_species_vcoef(beta):
    # every species falls at the speed of the smallest drop (r = 2 um) at
    # that radius; above it, the smaller exponents of the ice species make
    # them fall slower than drops of the same radius
    return tuple(8.0e3 * R1_CM ** (0.8 - b) for b in beta)


def gamma_spectrum_masses(x, rho, nu, rbar_cm, mtot):
    """Bin masses of a gamma spectrum in radius, n(r) ~ r^nu e^{-(nu+1)r/rbar},
    point-sampled on the mass grid (mass per bin ~ x r n(r)) and scaled to
    the total mass mtot; rows are points."""
    r = radius_cm(x, rho)[None, :]
    nu = np.asarray(nu, dtype=np.float64)[:, None]
    logm = np.log(x)[None, :] + (nu + 1.0) * np.log(r) - (nu + 1.0) * r / \
        rbar_cm
    logm -= logm.max(axis=1, keepdims=True)
    m = np.exp(logm)
    m *= (np.asarray(mtot, dtype=np.float64)[:, None] /
          m.sum(axis=1, keepdims=True))
    return m


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


# ---------------------------------------------------------------- config 1
def config1(npoints: int = 64, nsteps: int = 1800, dt: float = 1.0,
            s: int = 1, nbins: Optional[int] = None, b: float = 1500.0,
            lwc_g_m3: float = 1.0, rbar_cm: float = 1.0e-3) -> Workload:
    """Golovin kernel, one species, exponential start (identical points)."""
    B = nbins if nbins is not None else 33 * s
    x = bin_masses(B, s)
    xbar = 4.0 / 3.0 * np.pi * rbar_cm ** 3 * RHO_WATER
    L = lwc_g_m3 * 1e-6
    N0 = L / xbar
    n0 = N0 / xbar * np.exp(-x / xbar)
    M = x * x * n0 * (np.log(2.0) / s)
    M *= L / M.sum()
    N = np.ascontiguousarray(np.broadcast_to(M / x, (npoints, 1, B)))
    return Workload("golovin", B, 1, s, golovin_tables(B, s, b),
                    np.array([1000.0]), np.zeros((1, 1), np.int32), N,
                    np.full(npoints, 1000.0), dt, nsteps,
                    meta={"b": b, "N0": N0, "xbar": xbar, "L": L})


def constant_kernel(npoints=1, nsteps=1800, dt=1.0, s=1, C=1e-5,
                    lwc_g_m3=1.0, rbar_cm=1.0e-3) -> Workload:
    B = 33 * s
    x = bin_masses(B, s)
    xbar = 4.0 / 3.0 * np.pi * rbar_cm ** 3 * RHO_WATER
    L = lwc_g_m3 * 1e-6
    N0 = L / xbar
    n0 = N0 / xbar * np.exp(-x / xbar)
    M = x * x * n0 * (np.log(2.0) / s)
    M *= L / M.sum()
    N = np.ascontiguousarray(np.broadcast_to(M / x, (npoints, 1, B)))
    return Workload("constant", B, 1, s, constant_tables(B, C),
                    np.array([1000.0]), np.zeros((1, 1), np.int32), N,
                    np.full(npoints, 1000.0), dt, nsteps,
                    meta={"C": C, "N0": N0, "xbar": xbar, "L": L})


# ---------------------------------------------------------------- config 2
def config2(nx: int = 256, ny: int = 256, nz: int = 50, nsteps: int = 100,
            dt: float = 2.0, cloudy_frac: float = 0.15) -> Workload:
    """One GPU's patch of a thunderstorm domain, liquid only, 33 bins.
    Point index = (level * ny + y) * nx + x; pressure falls linearly with
    level from 1000 to 500 hPa."""
    rng = rng_for(2)
    B = 33
    P = nx * ny * nz
    x = bin_masses(B)
    cloudy = rng.random(P) < cloudy_frac
    idx = np.flatnonzero(cloudy)
    nc = idx.size
    nu = rng.uniform(2.0, 6.0, nc)
    lwc = _log_uniform(rng, 0.1, 3.0, nc)
    M = gamma_spectrum_masses(x, RHO_WATER, nu, 1.0e-3, lwc * 1e-6)
    N = np.zeros((P, 1, B))
    N[idx, 0, :] = M / x[None, :]
    level = np.arange(P) // (nx * ny)
    p = 1000.0 - 500.0 * level / max(nz - 1, 1)
    return Workload("thunderstorm_patch", B, 1, 1, liquid_tables(B),
                    P_LEVELS_3.copy(), np.zeros((1, 1), np.int32), N, p, dt,
                    nsteps, meta={"shape": (nz, ny, nx),
                                  "cloudy_frac": cloudy_frac})


# ---------------------------------------------------------------- config 3
def _multi_species_states(rng, x, rho, rbar, content_rng, present, npoints,
                          window):
    """Per species: gamma spectrum with its own mean radius and content;
    optional random active window [lo, hi] outside which the spectrum is
    zeroed (the content inside the window is kept as drawn)."""
    S = len(rho)
    B = x.size
    N = np.zeros((npoints, S, B))
    for a in range(S):
        sel = np.flatnonzero(present[:, a])
        n = sel.size
        nu = rng.uniform(2.0, 6.0, n)
        content = _log_uniform(rng, content_rng[a][0], content_rng[a][1], n)
        M = gamma_spectrum_masses(x, rho[a], nu, rbar[a], content * 1e-6)
        if window is not None:
            lo = rng.integers(window[0][0], window[0][1] + 1, n)
            hi = rng.integers(window[1][0], window[1][1] + 1, n)
            kk = np.arange(B)[None, :]
            M = np.where((kk >= lo[:, None]) & (kk <= hi[:, None]), M, 0.0)
        N[sel, a, :] = M / x[None, :]
    return N


def config3(npoints: int = 1 << 20, nsteps: int = 100,
            dt: float = 2.0) -> Workload:
    """Four species with 10 interacting pair kernels, random ice presence and
    uneven active-bin windows."""
    rng = rng_for(3)
    B, S = 33, 4
    x = bin_masses(B)
    present = np.ones((npoints, S), dtype=bool)
    present[:, 1:] = rng.random((npoints, 3)) < 0.3
    window = ((0, 5), (15, 32))
    N = _multi_species_states(rng, x, RHO_4, RBAR_4, CONTENT_4, present,
                              npoints, window)
    p = rng.uniform(500.0, 1000.0, npoints)
    tables = gravitational_tables(B, 1, RHO_4, BETA_4,
                                  multi_species_vcoef(BETA_4), P_LEVELS_3)
    return Workload("four_species", B, S, 1, tables, P_LEVELS_3.copy(),
                    PRODUCT_4.copy(), N, p, dt, nsteps,
                    meta={"species": SPECIES_4})


# The first four-species recipe: a liquid + crystal collision makes graupel,
# and every species carries the cloud-drop spectrum, all falling at the
# drop's speed at 100 um (smaller ice particles fall faster than drops of
# their radius).  Crystals collect droplets fast enough to over-demand
# their bins, so the positivity limiter fires at most points: the recipe
# exercises the limiter, the bench's four-species workload the method.
PRODUCT_4_GRAUPEL = np.array([[0, 3, 2, 3],
                              [3, 2, 2, 3],
                              [2, 2, 2, 3],
                              [3, 3, 3, 3]], dtype=np.int32)


def config3_limiter_heavy(npoints: int = 1 << 20, nsteps: int = 100,
                          dt: float = 2.0) -> Workload:
    """Config 3's species, kernels' construction, presence draws and active
    windows with the first recipe above (seed 8)."""
    rng = rng_for(8)
    B, S = 33, 4
    x = bin_masses(B)
    present = np.ones((npoints, S), dtype=bool)
    present[:, 1:] = rng.random((npoints, 3)) < 0.3
    N = _multi_species_states(rng, x, RHO_4, (RBAR_4[0],) * S,
                              (CONTENT_4[0],) * S, present, npoints,
                              ((0, 5), (15, 32)))
    p = rng.uniform(500.0, 1000.0, npoints)
    vcoef = tuple(8.0e3 * 100.0e-4 ** (0.8 - b) for b in BETA_4)
    tables = gravitational_tables(B, 1, RHO_4, BETA_4, vcoef, P_LEVELS_3)
    return Workload("four_species_limiter_heavy", B, S, 1, tables,
                    P_LEVELS_3.copy(), PRODUCT_4_GRAUPEL.copy(), N, p, dt,
                    nsteps, meta={"species": SPECIES_4})


# ------------------------------------------------- ice-crystal habits
# FSBM keeps the ice-crystal spectrum per habit (a second dimension of the
# crystal arrays, Sec. VI-C); here three habits (columns, plates,
# dendrites) are three species beside liquid, snow, graupel and hail.
SPECIES_7 = ("liquid", "ice_columns", "ice_plates", "ice_dendrites", "snow",
             "graupel", "hail")
BETA_7 = (0.8, 0.3, 0.25, 0.2, 0.4, 0.6, 0.7)
RHO_7 = (1.0, 0.9, 0.9, 0.5, 0.1, 0.4, 0.9)
RBAR_7 = (10.0e-4, 100.0e-4, 100.0e-4, 150.0e-4, 300.0e-4, 500.0e-4,
          800.0e-4)
CONTENT_7 = ((0.1, 3.0), (0.01, 0.1), (0.01, 0.1), (0.01, 0.1), (0.01, 0.5),
             (0.01, 1.0), (0.01, 0.5))
PRESENCE_7 = (1.0, 0.3, 0.3, 0.3, 0.3, 0.3, 0.1)


def _product_7():
    """Product species of the seven-species set (symmetric): drops rimed
    onto a particle keep its species (l + x -> x), two crystals of any
    habits and crystals with snow aggregate to snow, anything with graupel
    is graupel, anything with hail is hail."""
    S = 7
    P = np.zeros((S, S), dtype=np.int32)
    for a in range(S):
        for b in range(a, S):
            if a == 0:
                q = b
            elif b == 6:
                q = 6
            elif b == 5:
                q = 5
            else:
                q = 4          # habits and snow among themselves
            P[a, b] = P[b, a] = q
    return P


PRODUCT_7 = _product_7()


def config_habits(npoints: int = 1 << 18, nsteps: int = 100,
                  dt: float = 2.0) -> Workload:
    """Seven species: liquid, three ice-crystal habits, snow, graupel and
    hail on 33 doubling bins, 28 pair kernels; random presence per species
    and uneven active windows as in the four-species workload."""
    rng = rng_for(6)
    B, S = 33, 7
    x = bin_masses(B)
    present = rng.random((npoints, S)) < np.array(PRESENCE_7)[None, :]
    present[:, 0] = True
    N = _multi_species_states(rng, x, RHO_7, RBAR_7, CONTENT_7, present,
                              npoints, ((0, 5), (15, 32)))
    p = rng.uniform(500.0, 1000.0, npoints)
    tables = gravitational_tables(B, 1, RHO_7, BETA_7,
                                  multi_species_vcoef(BETA_7), P_LEVELS_3)
    return Workload("seven_species_habits", B, S, 1, tables,
                    P_LEVELS_3.copy(), PRODUCT_7.copy(), N, p, dt, nsteps,
                    meta={"species": SPECIES_7})


# ---------------------------------------------------------------- config 4
def _liquid_graupel():
    """Densities, exponents, mean radii and content ranges of the two
    species of the refined grids."""
    pick = (0, 3)
    return (tuple(RHO_4[a] for a in pick), tuple(BETA_4[a] for a in pick),
            tuple(RBAR_4[a] for a in pick), tuple(CONTENT_4[a] for a in pick))


def config4(nbins: int = 66, npoints: int = 262144, nsteps: int = 100,
            dt: float = 2.0, config_id: int = 4) -> Workload:
    """Liquid + graupel on a refined grid (66/132/264 bins, s = 2/4/8)."""
    s = {66: 2, 132: 4, 264: 8}[nbins]
    rng = rng_for(config_id)
    rho, beta, rbar, cont = _liquid_graupel()
    x = bin_masses(nbins, s)
    present = np.ones((npoints, 2), dtype=bool)
    N = _multi_species_states(rng, x, rho, rbar, cont, present, npoints,
                              None)
    p = rng.uniform(500.0, 1000.0, npoints)
    tables = gravitational_tables(nbins, s, rho, beta,
                                  multi_species_vcoef(beta), P_LEVELS_3)
    return Workload("liquid_graupel_%d" % nbins, nbins, 2, s, tables,
                    P_LEVELS_3.copy(), PRODUCT_2.copy(), N, p, dt, nsteps,
                    meta={"species": ("liquid", "graupel")})


# ---------------------------------------------------------------- config 5
def config5(npoints: int = 1 << 22, nsteps: int = 100, dt: float = 2.0,
            cloudy_frac: float = 0.10) -> List[Workload]:
    """Mixed-grid batch: each point is assigned to the 33-bin four-species
    grid (60%), the 66-bin or the 132-bin liquid+graupel grid (30%, 10%);
    10% of points are cloudy.  Returns one workload per grid."""
    rng = rng_for(5)
    grid = rng.choice(3, size=npoints, p=[0.6, 0.3, 0.1])
    cloudy = rng.random(npoints) < cloudy_frac
    out = []
    for g, (B, S, s) in enumerate(((33, 4, 1), (66, 2, 2), (132, 2, 4))):
        sel = np.flatnonzero(grid == g)
        n = sel.size
        x = bin_masses(B, s)
        cl = cloudy[sel]
        if S == 4:
            rho, beta, prod = RHO_4, BETA_4, PRODUCT_4
            rbar, cont = RBAR_4, CONTENT_4
            present = np.zeros((n, S), dtype=bool)
            present[:, 0] = cl
            present[:, 1:] = (rng.random((n, 3)) < 0.3) & cl[:, None]
            window = ((0, 5), (15, 32))
        else:
            rho, beta, rbar, cont = _liquid_graupel()
            prod = PRODUCT_2
            present = np.repeat(cl[:, None], 2, axis=1)
            window = None
        N = _multi_species_states(rng, x, rho, rbar, cont, present, n,
                                  window)
        p = rng.uniform(500.0, 1000.0, n)
        tables = gravitational_tables(B, s, rho, beta,
                                      multi_species_vcoef(beta), P_LEVELS_3)
        out.append(Workload("mixed_%d" % B, B, S, s, tables,
                            P_LEVELS_3.copy(), prod.copy(), N, p, dt, nsteps,
                            meta={"global_index": sel}))
    return out


def temperatures(npoints: int, seed: int = 0, lo: float = 185.0,
                 hi: float = 300.0):
    """Seeded per-point temperatures (K) for the collision gate: the
    current temperature uniform in [lo, hi] and the previous one within a
    few kelvin of it, so that points fall on both sides of both gate
    thresholds (193.15 K and 223.15 K).  Returns (t_old, t_now)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 2000 + seed))
    t_now = rng.uniform(lo, hi, npoints)
    t_old = t_now + rng.normal(0.0, 3.0, npoints)
    return t_old, t_now


def sample_active(w: Workload, n: int, seed: int = 0) -> np.ndarray:
    """Seeded subset of the cloudy point indices (sorted)."""
    act = np.flatnonzero(w.cloudy())
    if act.size <= n:
        return act
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 1000 + seed))
    return np.sort(rng.choice(act, size=n, replace=False))


# ------------------------------------------------------------ sedimentation
def fall_speed_cm_s(x, rho, beta, vcoef=None):
    """Fall speed [S][B] (cm/s) of every species and bin at 1000 hPa: the
    power law v = vcoef_a r^beta_a of the collection-kernel tables (r in
    cm; vcoef as in the multi-species tables unless given)."""
    if vcoef is None:
        vcoef = multi_species_vcoef(beta)
    return np.array([vcoef[a] * radius_cm(x, rho[a]) ** beta[a]
                     for a in range(len(rho))])


def _species_laws(w):
    """Densities and fall-speed exponents of a workload's species."""
    if w.name == "four_species":
        return RHO_4, BETA_4
    if w.name == "seven_species_habits":
        return RHO_7, BETA_7
    return tuple([RHO_WATER] * w.nspecies), tuple([0.8] * w.nspecies)


def sediment_geometry(w, nlev=None, column_major=False):
    """Columns of a workload for sedimentation: level-major patches
    ([nz][ny][nx], point = (level * ny + y) * nx + x) keep their grid;
    otherwise consecutive runs of nlev points form columns.  Layers thicken
    upward from 80 m to 140 m (1000 to 500 hPa over 50 levels spans about
    5.5 km); fall speeds follow the kernel tables' power laws, times
    (1000 / p)^0.4 at each point's pressure (the tables' air-density
    factor)."""
    shape = w.meta.get("shape") if w.meta else None
    if shape is not None and not column_major:
        nz, ny, nx = shape
        nlev, ncols = nz, nx * ny
        col_stride, lev_stride = 1, nx * ny
    else:
        if nlev is None:
            raise ValueError("nlev is needed for a workload without a grid")
        ncols = w.npoints // nlev
        col_stride, lev_stride = nlev, 1
    lev = np.arange(nlev)
    dz_cm = 8000.0 + 6000.0 * lev / max(nlev - 1, 1)
    rho, beta = _species_laws(w)
    x = bin_masses(w.nbins, w.s, w.x1_g)
    v = fall_speed_cm_s(x, rho, beta)
    pts = (np.arange(ncols)[:, None] * col_stride +
           lev[None, :] * lev_stride)
    vfac = (1000.0 / w.p[pts]) ** 0.4
    return {"ncols": ncols, "nlev": nlev, "col_stride": col_stride,
            "lev_stride": lev_stride, "dz_cm": dz_cm,
            "v_cm_s": np.ascontiguousarray(v), "vfac": np.ascontiguousarray(vfac),
            "max_courant_per_s": float(v.max() * vfac.max() / dz_cm.min())}


# ------------------------------------------------------------ condensation
def condensation_inputs(w: Workload, seed: int = 0):
    """Seeded per-point supersaturation (fraction) and growth coefficient
    G (cm^2/s) for condensation of a workload's first species: 70 % of the
    points growing, s ~ U[0, 1 %] (in-cloud values), 30 % evaporating,
    |s| log-uniform in [0.1 %, 10 %] (sub-saturated air);
    G = 1e-6 (1000 / p)^0.2 U[0.9, 1.1] (about 100 um^2/s near 10 C, rising
    with the vapour diffusivity as the pressure falls).  Returns
    (ssat, gcoef), float64 [npoints]."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 3000 + seed))
    P = w.npoints
    grow = rng.random(P) < 0.7
    ssat = np.where(grow, rng.uniform(0.0, 0.01, P),
                    -_log_uniform(rng, 1e-3, 0.1, P))
    gcoef = 1e-6 * (1000.0 / w.p) ** 0.2 * rng.uniform(0.9, 1.1, P)
    return np.ascontiguousarray(ssat), np.ascontiguousarray(gcoef)


# ---------------------------------------------------------------- breakup
def breakup_tables(nbins: int, s: int = 1, x1: float = X1_G,
                   frag_ratio: float = 8.0):
    """Spontaneous-breakup inputs of the liquid on a grid: the rate per bin,
    P(D) = 2.94e-7 exp(34 D) s^-1 with D the drop diameter in cm (the
    exponential form of Komabayasi, Gonda and Isono 1964; the smallest bin
    does not break), and the fragment table: a broken drop of bin l gives
    fragments in the bins k < l with numbers proportional to
    exp(-x_k / xbar), xbar = x_l / frag_ratio, scaled so that their mass is
    x_l.  Returns (rate [B], fragments [B][B])."""
    x = bin_masses(nbins, s, x1)
    D = 2.0 * radius_cm(x, RHO_WATER)
    rate = 2.94e-7 * np.exp(34.0 * D)
    rate[0] = 0.0
    Q = np.zeros((nbins, nbins))
    for l in range(1, nbins):
        w = np.exp(-x[:l] / (x[l] / frag_ratio))
        Q[l, :l] = w * (x[l] / float(w @ x[:l]))
    return np.ascontiguousarray(rate), np.ascontiguousarray(Q)
