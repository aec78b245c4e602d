/*
 * fsbm_oracle.c -- plain FP64 CPU oracle of the FSBM collision-coalescence
 * step.  TEST INFRASTRUCTURE ONLY (see fsbm_oracle.h): it is loaded by the
 * tests, the smoke check and the benchmark's CPU-baseline leg, never by the
 * GPU library.
 *
 * Written for a reader checking it against the method by eye: one point at a
 * time, the pair loop in one canonical order, no blocking, no fusion, no
 * precomputed products beyond the bin grid and the (k, c) target tables.
 *
 * Sources followed:
 *  - Sec. III, eq. (1): one equation per bin and particle type, the collision
 *    term being one of the process tendencies; 33 bins per type.
 *  - Sec. III (the hot routine is named after Bott's flux method) and
 *    Bott (1998, J. Atmos. Sci. 55, 2284): mass removed from both colliding
 *    bins, the merged mass placed into the bin below x_i + x_j and a fraction
 *    moved on to the next bin with an exponential sub-bin profile.
 *  - Sec. VI-A, "Lookup optimization": collection kernels tabulated per pair
 *    of particle types at two (here: L) pressure levels and interpolated
 *    linearly for the point's pressure; cost quadratic in the bin count.
 *  - Sec. VI-B: the collision call is made only for points whose predicate
 *    holds (here: the point holds mass).
 * The paper leaves the collision arithmetic open; each choice taken here
 * is a reading, marked [R#] where it shapes the arithmetic below.
 *
 * Pins: the tests check this code against closed forms of the collection
 * equation (constant and Golovin kernels), hand-worked steps in exact
 * binary fractions, conservation, positivity, number decrease and the
 * refinement ladder.  Parity unpinned: the exact form of the flux fraction
 * [R3], the empty-neighbour guard value [R4], the off-grid rule [R6] and
 * the species product map [R11] are fixed by these readings alone; no
 * source in reach gives their values, and the pins above constrain the
 * method as a whole, not these constants.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include "fsbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* [R4] guard for an empty neighbour bin: x1 >= ln(1e-60). */
#define X1_FLOOR (-60.0 * 2.302585092994045684)
/* [R5] relative tolerance that turns an exact hit x_i + x_j == x_k into c=0 */
#define HIT_TOL 1e-12

typedef struct {
  const fsbm_oracle_desc *d;
  int B, S, L, npairs_species;
  double *x;     /* [B] */
  int32_t *kt;   /* [B][B] target bin, -1 = leaves the grid */
  double *ct;    /* [B][B] Courant number of the target */
} ctx_t;

static int species_pair_index(int S, int a, int b) {
  /* pairs (0,0),(0,1),...,(0,S-1),(1,1),...: row a starts after
     S + (S-1) + ... + (S-a+1) entries */
  return a * S - (a * (a - 1)) / 2 + (b - a);
}

static int check_desc(const fsbm_oracle_desc *d) {
  if (!d || d->nbins < 2 || d->nspecies < 1 || d->nspecies > 8 ||
      d->nlevels < 1 || d->s < 1 || !(d->x1_g > 0.0) || !d->tables ||
      !d->p_levels || !d->product || d->order < 0 || d->order > 1 ||
      !(d->theta >= 0.0))
    return -1;
  if (d->order == 1 && d->nspecies != 1) return -1; /* [R16]: one species */
  for (int l = 0; l + 1 < d->nlevels; ++l)
    if (!(d->p_levels[l] > d->p_levels[l + 1])) return -1;
  for (int a = 0; a < d->nspecies; ++a)
    for (int b = 0; b < d->nspecies; ++b) {
      int P = d->product[a * d->nspecies + b];
      if (P < 0 || P >= d->nspecies) return -1;
      if (P != d->product[b * d->nspecies + a]) return -1;
    }
  return 0;
}

/* Bin masses: x_k = x_1 * 2^(k/s), built with ldexp so that x_{k+s} = 2 x_k
   holds exactly [R5]. */
static void build_grid(const fsbm_oracle_desc *d, double *x) {
  for (int k = 0; k < d->nbins; ++k) {
    double frac = pow(2.0, (double)(k % d->s) / (double)d->s);
    x[k] = ldexp(d->x1_g * frac, k / d->s);
  }
}

/* Mass of the (possibly virtual) bin k >= B on the same grid. */
static double grid_mass(const fsbm_oracle_desc *d, int k) {
  double frac = pow(2.0, (double)(k % d->s) / (double)d->s);
  return ldexp(d->x1_g * frac, k / d->s);
}

/* Target tables: k_ij = largest k with x_k <= (x_i + x_j)(1 + tol); a pair
   whose k reaches B leaves the grid and is skipped [R6]; for k <= B-2 the
   Courant number is the position of x_i + x_j inside [x_k, x_{k+1}]. */
static void build_targets(const fsbm_oracle_desc *d, const double *x,
                          int32_t *kt, double *ct) {
  int B = d->nbins;
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j) {
      double sum = x[i] + x[j];
      int k = 0;
      while (grid_mass(d, k + 1) <= sum * (1.0 + HIT_TOL)) ++k;
      double c = 0.0;
      if (k >= B) {
        k = -1;
      } else if (k <= B - 2) {
        c = (sum - x[k]) / (x[k + 1] - x[k]);
        if (c < 0.0) c = 0.0;
        if (c > 1.0) c = 1.0;
      }
      kt[i * B + j] = k;
      ct[i * B + j] = c;
    }
}

/* Flux fraction of the merged mass that moves from bin k to bin k+1 [R3]:
   the sub-bin profile is exp(x1 * t) on t in [-1/2, 1/2] and the fraction is
   the integral of that profile over the top c of the bin,
       f = int_{1/2-c}^{1/2} exp(x1 t) dt = exp((1/2 - c) x1) expm1(c x1) / x1,
   which tends to c as x1 -> 0.  The result is clamped to [0, 1]. */
double fsbm_oracle_flux_fraction(double c, double x1) {
  double f;
  if (c == 0.0) {
    f = 0.0;
  } else if (x1 == 0.0) {
    f = c;
  } else if (x1 > 700.0) {
    /* f grows with x1 for x1 >= 0 and already exceeds 1 here for every
       c > 1e-150, so the clamp below decides; this branch only avoids an
       inf*0 in the formula. */
    f = 1.0;
  } else {
    f = exp((0.5 - c) * x1) * expm1(c * x1) / x1;
  }
  if (f < 0.0) f = 0.0;
  if (f > 1.0) f = 1.0;
  return f;
}

/* Pressure bracket [R10]: clamp p into [p_{L-1}, p_0], take the first level
   pair with p_l >= p >= p_{l+1}, weight w of level l. */
static void pressure_bracket(const fsbm_oracle_desc *d, double p, int *l_out,
                             double *w_out) {
  int L = d->nlevels;
  if (L == 1) {
    *l_out = 0;
    *w_out = 1.0;
    return;
  }
  const double *pl = d->p_levels;
  if (p > pl[0]) p = pl[0];
  if (p < pl[L - 1]) p = pl[L - 1];
  int l = 0;
  while (l < L - 2 && !(pl[l] >= p && p >= pl[l + 1])) ++l;
  *l_out = l;
  *w_out = (p - pl[l + 1]) / (pl[l] - pl[l + 1]);
}

/* K^{ab}_{ij}(p) = K_{l+1} + (K_l - K_{l+1}) w, the form of the lookup
   expression shown in Sec. VI-A; one level means no interpolation. */
static double kernel_entry(const fsbm_oracle_desc *d, int ab, int l, double w,
                           int i, int j) {
  int B = d->nbins, L = d->nlevels;
  const double *t = d->tables + (size_t)ab * L * B * B;
  if (L == 1) return t[(size_t)i * B + j];
  double k_l = t[(size_t)l * B * B + (size_t)i * B + j];
  double k_l1 = t[(size_t)(l + 1) * B * B + (size_t)i * B + j];
  return k_l1 + (k_l - k_l1) * w;
}

double fsbm_oracle_kernel_at(const fsbm_oracle_desc *d, double p, int32_t a,
                             int32_t b, int32_t i, int32_t j) {
  if (check_desc(d)) return NAN;
  if (a > b) {
    int32_t t = a;
    a = b;
    b = t;
    t = i;
    i = j;
    j = t;
  }
  int l;
  double w;
  pressure_bracket(d, p, &l, &w);
  return kernel_entry(d, species_pair_index(d->nspecies, a, b), l, w, i, j);
}

/* One bin pair's net contributions after merging entries that hit the same
   bin.  Up to four (bin, amount) entries, in the order (a,i), (b,j), (P,k),
   (P,k+1); returns their number. */
typedef struct {
  int n;
  int bin[4];
  double amt[4];
} contrib_t;

static void add_entry(contrib_t *c, int bin, double amt) {
  for (int e = 0; e < c->n; ++e)
    if (c->bin[e] == bin) {
      c->amt[e] += amt;
      return;
    }
  c->bin[c->n] = bin;
  c->amt[c->n] = amt;
  c->n++;
}

/* S4 for one pair.  Mt: masses with inactive bins set to zero; N: numbers.
   Returns 0 when the pair contributes nothing. */
static int pair_contrib(const ctx_t *cx, const double *Mt, const double *N,
                        int a, int i, int b, int j, double K, double dt,
                        contrib_t *out) {
  const int B = cx->B;
  int k = cx->kt[i * B + j];
  out->n = 0;
  if (k < 0) return 0; /* merged mass leaves the grid [R6] */
  double C = dt * K * N[a * B + i] * N[b * B + j];
  if (a == b && i == j) C *= 0.5; /* each unordered pair counted once [R7] */
  if (C == 0.0) return 0;
  double A = C * cx->x[i];
  double Bm = C * cx->x[j];
  double Sm = A + Bm;
  int P = cx->d->product[a * cx->S + b];
  double F = 0.0;
  if (k <= B - 2) {
    double r = Mt[P * B + k + 1] / (Mt[P * B + k] + Sm);
    double x1 = log(r);
    if (!(x1 >= X1_FLOOR)) x1 = X1_FLOOR; /* also catches log(0) = -inf */
    double f = fsbm_oracle_flux_fraction(cx->ct[i * B + j], x1);
    F = f * Sm;
  }
  /* Contributions to the same bin are combined first [S4].  When the
     merged mass lands in one of the two source bins, that bin's combined
     contribution is formed directly as the other source's collided mass
     minus the flux, not as -Bm + ((A + Bm) - F): the rounding of A + Bm
     alone is up to u Bm / 2, far above A - F when a large particle
     collects a small one. */
  const int qa = a * B + i, qb = b * B + j, qk = P * B + k;
  if (qk == qb && qk != qa) {
    add_entry(out, qa, -A);
    add_entry(out, qb, A - F);
  } else if (qk == qa && qk != qb) {
    add_entry(out, qa, Bm - F);
    add_entry(out, qb, -Bm);
  } else {
    add_entry(out, qa, -A);
    add_entry(out, qb, -Bm);
    add_entry(out, qk, Sm - F);
  }
  if (k <= B - 2) add_entry(out, qk + 1, F);
  return 1;
}

typedef struct {
  double *M, *Mt, *G, *Ls, *D, *sig;
  unsigned char *act;
} work_t;

/* Visit every pair in the canonical order [S4]: species pairs (a <= b)
   lexicographic, then i ascending, then j ascending (j >= i when a == b);
   a pair is evaluated only if both of its bins are active.
   mode 0: accumulate G, L and the demand D;  mode 1: accumulate G, L with
   every pair scaled by its limiter factor (the minimum sigma over the bins
   where the pair's net is negative) [R9]. */
static void pair_pass(const ctx_t *cx, const double *N, int l, double w,
                      double dt, work_t *wk, int mode) {
  const int B = cx->B, S = cx->S;
  contrib_t ct;
  for (int a = 0; a < S; ++a)
    for (int b = a; b < S; ++b) {
      int ab = species_pair_index(S, a, b);
      for (int i = 0; i < B; ++i) {
        if (!wk->act[a * B + i]) continue;
        for (int j = (a == b ? i : 0); j < B; ++j) {
          if (!wk->act[b * B + j]) continue;
          double K = kernel_entry(cx->d, ab, l, w, i, j);
          if (!pair_contrib(cx, wk->Mt, N, a, i, b, j, K, dt, &ct)) continue;
          double scale = 1.0;
          if (mode == 1)
            for (int e = 0; e < ct.n; ++e)
              if (ct.amt[e] < 0.0 && wk->sig[ct.bin[e]] < scale)
                scale = wk->sig[ct.bin[e]];
          for (int e = 0; e < ct.n; ++e) {
            double v = ct.amt[e] * scale;
            if (v > 0.0) {
              wk->G[ct.bin[e]] += v;
            } else if (v < 0.0) {
              wk->Ls[ct.bin[e]] += -v;
              if (mode == 0) wk->D[ct.bin[e]] += -v;
            }
          }
        }
      }
    }
}

/* One time step of one point (S1-S6).  Returns 1 if the limiter fired.
   lim_bins (NULL or [S*B]): set to 1 for every bin whose limiter factor
   sigma is below 1 in this step. */
static int step_point(const ctx_t *cx, double *N, double p, double dt,
                      work_t *wk, unsigned char *lim_bins) {
  const int B = cx->B, S = cx->S, n = S * B;
  /* S1: masses and the point total, species then bins ascending. */
  double Mtot = 0.0;
  for (int q = 0; q < n; ++q) {
    wk->M[q] = N[q] * cx->x[q % B];
    Mtot += wk->M[q];
  }
  if (Mtot == 0.0) return 0;
  /* S2: activity [R8]. */
  double thr = cx->d->theta * Mtot;
  for (int q = 0; q < n; ++q) {
    wk->act[q] = (wk->M[q] > 0.0 && wk->M[q] >= thr);
    wk->Mt[q] = wk->act[q] ? wk->M[q] : 0.0;
    wk->G[q] = wk->Ls[q] = wk->D[q] = 0.0;
    wk->sig[q] = 1.0;
  }
  /* S3: pressure bracket of this point. */
  int l;
  double w;
  pressure_bracket(cx->d, p, &l, &w);
  /* S4 + S5 detection. */
  pair_pass(cx, N, l, w, dt, wk, 0);
  int limited = 0;
  for (int q = 0; q < n; ++q)
    if (wk->D[q] > wk->M[q]) limited = 1;
  if (limited) {
    /* S5: sigma per bin, then a second pass with per-pair scaling. */
    for (int q = 0; q < n; ++q) {
      wk->sig[q] = 1.0;
      if (wk->D[q] > wk->M[q]) {
        wk->sig[q] = wk->M[q] / wk->D[q];
        if (lim_bins) lim_bins[q] = 1;
      }
      wk->G[q] = wk->Ls[q] = 0.0;
    }
    pair_pass(cx, N, l, w, dt, wk, 1);
  }
  /* S6: update in mass, clamp negative round-off, back to numbers. */
  for (int q = 0; q < n; ++q) {
    double Mn = wk->M[q] + (wk->G[q] - wk->Ls[q]);
    if (Mn < 0.0) Mn = 0.0;
    N[q] = Mn / cx->x[q % B];
  }
  return limited;
}

/* One time step of one point in Bott's original, sequential form [R16]
   (one species): the pairs are taken one after another in the canonical
   order (i ascending, then j = i..B-1 ascending) and each pair moves mass
   in place, so a pair sees every change made by the pairs before it.
   Per pair (i, j) whose bins are both active with their current masses:
     C  = dt K_ij(p) N_i N_j  (1/2 of it when i == j)     collisions per cm^3
     A  = C x_i leaves bin i, Bm = C x_j leaves bin j, Sm = A + Bm merges
     into bin k = k_ij, and the flux F = f(c_ij, x1) Sm moves on to k+1 with
     x1 = ln(M_{k+1} / M_k'), M_k' the content of bin k after the removals
     and the merge (the profile of the simultaneous form [R3, R4]).
   Positivity without a second pass, by caps on the bins that lose mass:
     C <= N_i (C <= N_i / 2 when i == j): bin i gives at most what it holds;
     C <= N_j when the merged mass does not land in bin j (when it does, the
     collector bin keeps its particles, which may collide many times);
     F <= M_k': the flux moves at most what bin k then holds.
   A bin whose cap applied is left with exactly nothing, the value of
   M - (M / x) x in exact arithmetic: a rounding residue of either sign
   would keep or drop the bin from the later pairs of the step, and a pair
   (i, j) moves 2^(j-i) times bin i's mass in bin j, so residues would be
   amplified by up to 2^(B-1).  Returns the number of capped pairs; sets
   lim_bins[q] (NULL or [B]) for every bin a cap emptied. */
static int step_point_seq(const ctx_t *cx, double *N, double p, double dt,
                          double *M, unsigned char *lim_bins) {
  const int B = cx->B;
  const double *x = cx->x;
  double Mtot = 0.0;
  for (int q = 0; q < B; ++q) {
    M[q] = N[q] * x[q];
    Mtot += M[q];
  }
  if (Mtot == 0.0) return 0;
  /* activity [R8] with the current masses against the step's total */
  const double thr = cx->d->theta * Mtot;
  int l;
  double w;
  pressure_bracket(cx->d, p, &l, &w);
  int capped = 0;
  for (int i = 0; i < B; ++i)
    for (int j = i; j < B; ++j) {
      if (!(M[i] > 0.0 && M[i] >= thr && M[j] > 0.0 && M[j] >= thr))
        continue;
      const int k = cx->kt[i * B + j];
      if (k < 0) continue; /* [R6] */
      const double K = kernel_entry(cx->d, 0, l, w, i, j);
      const double Ni = M[i] / x[i], Nj = M[j] / x[j];
      double C = dt * K * Ni * Nj;
      double cap = Ni;
      if (i == j) {
        C *= 0.5; /* [R7] */
        cap = 0.5 * Ni;
      } else if (k != j && Nj < cap) {
        cap = Nj;
      }
      int hit = 0;
      if (C > cap) {
        C = cap;
        hit = 1;
      }
      if (C == 0.0) continue;
      const double A = C * x[i], Bm = C * x[j], Sm = A + Bm;
      /* removals; the target's content after them and the merged mass.  When
         the target is the partner bin j, its content is formed as M_j + A
         (the same value as (M_j - Bm) + Sm without the rounding of the large
         Bm twice). */
      double Mk;
      int emptied_i = 0, emptied_j = 0;
      if (i == j) {
        emptied_i = hit;
        M[i] = hit ? 0.0 : M[i] - Sm;
        Mk = M[k] + Sm;
      } else if (k == j) {
        emptied_i = hit;
        M[i] = hit ? 0.0 : M[i] - A;
        Mk = M[j] + A;
      } else {
        emptied_i = hit && C == Ni;
        emptied_j = hit && C == Nj;
        M[i] = emptied_i ? 0.0 : M[i] - A;
        M[j] = emptied_j ? 0.0 : M[j] - Bm;
        Mk = M[k] + Sm;
      }
      if (lim_bins) {
        if (emptied_i) lim_bins[i] = 1;
        if (emptied_j) lim_bins[j] = 1;
      }
      double F = 0.0;
      if (k <= B - 2) {
        double x1 = log(M[k + 1] / Mk);
        if (!(x1 >= X1_FLOOR)) x1 = X1_FLOOR; /* [R4]; also log(0) */
        F = fsbm_oracle_flux_fraction(cx->ct[i * B + j], x1) * Sm;
        if (F > Mk) {
          F = Mk;
          hit = 1;
          if (lim_bins) lim_bins[k] = 1;
        }
        M[k + 1] += F;
      }
      M[k] = Mk - F;
      capped += hit;
    }
  /* back to numbers; negative round-off clamped as in S6 */
  for (int q = 0; q < B; ++q) N[q] = (M[q] < 0.0 ? 0.0 : M[q]) / x[q];
  return capped;
}

static void point_totals(const ctx_t *cx, const double *N, double *m,
                         double *num) {
  const int B = cx->B, n = cx->S * B;
  double sm = 0.0, sn = 0.0;
  for (int q = 0; q < n; ++q) {
    sm += N[q] * cx->x[q % B];
    sn += N[q];
  }
  *m = sm;
  *num = sn;
}

int fsbm_oracle_grid(const fsbm_oracle_desc *d, double *x) {
  if (check_desc(d) || !x) return -1;
  build_grid(d, x);
  return 0;
}

int fsbm_oracle_targets(const fsbm_oracle_desc *d, int32_t *k, double *c) {
  if (check_desc(d) || !k || !c) return -1;
  double *x = (double *)malloc(sizeof(double) * d->nbins);
  if (!x) return -1;
  build_grid(d, x);
  build_targets(d, x, k, c);
  free(x);
  return 0;
}

int fsbm_oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* The collision call of a point is made only where the point is warm
   enough: the main loop over grid points (Sec. III, its listing) calls the
   collision routine inside a test of the previous temperature against
   193.15 K and, nested in it, of the current one against 223.15 K, both
   strict.  A missing array (NULL) passes its test. */
#define T_OLD_MIN 193.15
#define T_COLL_MIN 223.15

static int point_passes_gate(const double *t_old, const double *t_now,
                             int64_t pt) {
  if (t_old && !(t_old[pt] > T_OLD_MIN)) return 0;
  if (t_now && !(t_now[pt] > T_COLL_MIN)) return 0;
  return 1;
}

int fsbm_oracle_run(const fsbm_oracle_desc *d, double *N, const double *p,
                    int64_t npoints, double dt, int32_t nsteps,
                    double *mass_before, double *mass_after,
                    double *num_before, double *num_after,
                    int64_t *limiter_steps, int32_t *limiter_per_point,
                    unsigned char *limited_bins, int32_t nthreads) {
  return fsbm_oracle_run_gated(d, N, p, NULL, NULL, npoints, dt, nsteps,
                               mass_before, mass_after, num_before,
                               num_after, limiter_steps, limiter_per_point,
                               limited_bins, nthreads);
}

int fsbm_oracle_run_gated(const fsbm_oracle_desc *d, double *N,
                          const double *p, const double *t_old,
                          const double *t_now, int64_t npoints, double dt,
                          int32_t nsteps, double *mass_before,
                          double *mass_after, double *num_before,
                          double *num_after, int64_t *limiter_steps,
                          int32_t *limiter_per_point,
                          unsigned char *limited_bins, int32_t nthreads) {
  if (check_desc(d) || npoints < 0 || nsteps < 0 || !(dt > 0.0) ||
      !isfinite(dt))
    return -1;
  if (npoints > 0 && (!N || !p)) return -1;
  ctx_t cx;
  cx.d = d;
  cx.B = d->nbins;
  cx.S = d->nspecies;
  cx.L = d->nlevels;
  cx.npairs_species = d->nspecies * (d->nspecies + 1) / 2;
  cx.x = (double *)malloc(sizeof(double) * cx.B);
  cx.kt = (int32_t *)malloc(sizeof(int32_t) * cx.B * cx.B);
  cx.ct = (double *)malloc(sizeof(double) * cx.B * cx.B);
  if (!cx.x || !cx.kt || !cx.ct) {
    free(cx.x);
    free(cx.kt);
    free(cx.ct);
    return -1;
  }
  build_grid(d, cx.x);
  build_targets(d, cx.x, cx.kt, cx.ct);
  const int n = cx.S * cx.B;
  int64_t lim_total = 0;
  int failed = 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(+ : lim_total) \
    reduction(| : failed)
#endif
  {
    work_t wk;
    double *buf = (double *)malloc(sizeof(double) * 6 * n);
    wk.act = (unsigned char *)malloc(n);
    if (!buf || !wk.act) {
      failed = 1;
    } else {
      wk.M = buf;
      wk.Mt = buf + n;
      wk.G = buf + 2 * n;
      wk.Ls = buf + 3 * n;
      wk.D = buf + 4 * n;
      wk.sig = buf + 5 * n;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
      for (int64_t pt = 0; pt < npoints; ++pt) {
        double *Np = N + pt * n;
        double m0, n0;
        point_totals(&cx, Np, &m0, &n0);
        if (mass_before) mass_before[pt] = m0;
        if (num_before) num_before[pt] = n0;
        int32_t lim_pt = 0;
        unsigned char *lb = limited_bins ? limited_bins + pt * n : NULL;
        if (lb) memset(lb, 0, (size_t)n);
        const int steps = point_passes_gate(t_old, t_now, pt) ? nsteps : 0;
        for (int st = 0; st < steps; ++st)
          lim_pt += d->order == 1
                        ? step_point_seq(&cx, Np, p[pt], dt, wk.M, lb)
                        : step_point(&cx, Np, p[pt], dt, &wk, lb);
        lim_total += lim_pt;
        if (limiter_per_point) limiter_per_point[pt] = lim_pt;
        if (mass_after || num_after) {
          point_totals(&cx, Np, &m0, &n0);
          if (mass_after) mass_after[pt] = m0;
          if (num_after) num_after[pt] = n0;
        }
      }
    }
    free(buf);
    free(wk.act);
  }
  free(cx.x);
  free(cx.kt);
  free(cx.ct);
  if (limiter_steps) *limiter_steps = lim_total;
  return failed ? -1 : 0;
}
