/*
 * fsbm_oracle_break.c -- plain FP64 CPU oracle of spontaneous breakup of a
 * drop spectrum on the fixed mass grid.  TEST INFRASTRUCTURE ONLY (see
 * fsbm_oracle.h): loaded by the tests, the smoke check and the benchmark's
 * CPU-baseline leg, never by the GPU library; it shares no code with it.
 *
 * The paper lists breakup among the process terms of the bin equation
 * (Sec. III, eq. (1)) without giving its form.  Readings taken here
 * ([R26]-[R28]), after the linear breakup equation of Srivastava (1971)
 * with a breakup probability per unit time of the kind fitted by
 * Komabayasi, Gonda and Isono (1964):
 *  [R26] a drop of bin l breaks at a rate P_l (s^-1, per bin, given) into
 *        Q[l][k] fragments in each smaller bin k < l (a given table with
 *        Q[l][k] = 0 for k >= l, mass-balanced by the caller:
 *        sum_k Q[l][k] x_k = x_l); the smallest bin does not break;
 *        dN_k/dt = -P_k N_k + sum_{l>k} P_l N_l Q[l][k];
 *  [R27] over a step dt, the share of bin l's drops that break is
 *        b_l = 1 - exp(-P_l dt) (the exact solution of the loss term
 *        alone: fragments do not break again within the step), so
 *        N'_k = (N_k - b_k N_k) + sum_{l>k} (b_l N_l) Q[l][k], the sum
 *        taken in ascending l;
 *  [R28] b_l is computed as -expm1(-P_l dt) (accurate for small P dt).
 * With these readings the liquid mass is kept to the fragment table's
 * own balance, N stays >= 0, the number never falls, P = 0 is the
 * identity, and as dt -> 0 at fixed n dt the result tends to the exact
 * solution exp(T M) N_0 of the linear system (first order in dt).  The
 * tests pin these.
 *
 * N: [npoints][B] number per cm^3 per bin, in place; rate_per_s: [B];
 * fragments: [B][B], row l = the fragments of one drop of bin l.
 */
#include "fsbm_oracle.h"

#include <math.h>
#include <stdlib.h>

int fsbm_oracle_breakup(int32_t nbins, int64_t npoints, double *N,
                        const double *rate_per_s, const double *fragments,
                        double dt, int32_t nsteps) {
  if (nbins < 2 || npoints < 0 || nsteps < 0 || !(dt > 0.0) ||
      !isfinite(dt) || !rate_per_s || !fragments || (npoints > 0 && !N))
    return -1;
  const int B = nbins;
  for (int l = 0; l < B; ++l) {
    if (!(rate_per_s[l] >= 0.0) || !isfinite(rate_per_s[l])) return -1;
    for (int k = 0; k < B; ++k) {
      const double q = fragments[(size_t)l * B + k];
      if (!(q >= 0.0) || !isfinite(q) || (k >= l && q != 0.0)) return -1;
    }
  }
  double *b = (double *)malloc(sizeof(double) * B);
  double *L = (double *)malloc(sizeof(double) * B);
  if (!b || !L) {
    free(b);
    free(L);
    return -1;
  }
  b[0] = 0.0; /* [R26] the smallest bin does not break */
  for (int l = 1; l < B; ++l) b[l] = -expm1(-rate_per_s[l] * dt); /* [R28] */
  for (int64_t pt = 0; pt < npoints; ++pt) {
    double *Np = N + pt * B;
    for (int32_t st = 0; st < nsteps; ++st) {
      for (int l = 0; l < B; ++l) L[l] = b[l] * Np[l]; /* [R27] broken */
      for (int k = 0; k < B; ++k) {
        double v = Np[k] - L[k];
        for (int l = k + 1; l < B; ++l)
          v += L[l] * fragments[(size_t)l * B + k];
        Np[k] = v;
      }
    }
  }
  free(b);
  free(L);
  return 0;
}
