/*
 * fsbm_oracle_cond.c -- plain FP64 CPU oracle of condensation and
 * evaporation of a drop spectrum on the fixed mass grid.  TEST
 * INFRASTRUCTURE ONLY (see fsbm_oracle.h): loaded by the tests, the smoke
 * check and the benchmark's CPU-baseline leg, never by the GPU library; it
 * shares no code with it.
 *
 * The paper lists condensation/evaporation among the process terms of the
 * bin equation (Sec. III, eq. (1)), calls it from the main loop over grid
 * points (the condensation routines of the Sec. III listing) and names it
 * as the next part to offload (Sec. VIII), without giving its form.
 * Readings taken here ([R22]-[R25]), from published formulations:
 *  [R22] diffusional growth of a drop at a prescribed supersaturation s
 *        (fraction, s < 0 evaporates) with a growth coefficient G (cm^2/s)
 *        per point, curvature and solute terms left out: r dr/dt = G s
 *        (Rogers and Yau 1989, ch. 7), so over a step r^2 grows by
 *        2 G s dt exactly; the vapour and heat budgets (the feedback of
 *        s and G) are the caller's;
 *  [R23] every drop of bin k (mass x_k, radius r_k of a sphere of density
 *        rho) moves to the mass x' = (4 pi rho / 3) (r_k^2 + 2 G s dt)^(3/2);
 *        its number is then shared between the two grid bins around x'
 *        so that number and mass are both kept: N (1 - phi) to bin j and
 *        N phi to bin j+1, x_j <= x' < x_{j+1}, phi = (x' - x_j) /
 *        (x_{j+1} - x_j) (the two-moment remapping of Kovetz and Olund
 *        1969); contributions are added in ascending source bin order;
 *  [R24] a drop whose r^2 would fall to 0 or below, or whose new mass is
 *        below the smallest bin, evaporates completely: its number leaves
 *        the spectrum and its mass x_k is reported as evaporated;
 *  [R25] a drop that grows to the last bin's mass or beyond is kept in the
 *        last bin (the grid's end; the liquid gain is then x_{B-1} - x_k
 *        per drop).
 * With these readings number is conserved except for [R24] removals, the
 * liquid mass changes by exactly sum N (x' - x_k) away from the grid's
 * ends, s = 0 is the identity, and a drop landing on a grid point moves
 * there whole.  The tests pin these and a refinement ladder against the
 * exact r^2 law of a monodisperse population.
 *
 * Grid: x_k = x1 2^(k/s_grid) as in the collision oracle (doubling exact).
 * N: [npoints][B] number per cm^3 per bin, in place; ssat, gcoef: [npoints];
 * evaporated: [npoints] g cm^-3 added to (or NULL).
 */
#include "fsbm_oracle.h"

#include <math.h>
#include <stdlib.h>

#define COND_PI 3.14159265358979323846

static double cond_grid_mass(double x1, int s, int k) {
  return ldexp(x1 * pow(2.0, (double)(k % s) / (double)s), k / s);
}

int fsbm_oracle_condense(int32_t nbins, int32_t s_grid, double x1_g,
                         double rho_g_cm3, int64_t npoints, double *N,
                         const double *ssat, const double *gcoef_cm2_s,
                         double dt, int32_t nsteps, double *evaporated) {
  if (nbins < 2 || s_grid < 1 || !(x1_g > 0.0) || !(rho_g_cm3 > 0.0) ||
      npoints < 0 || nsteps < 0 || !(dt > 0.0) || !isfinite(dt) ||
      (npoints > 0 && (!N || !ssat || !gcoef_cm2_s)))
    return -1;
  const int B = nbins;
  double *x = (double *)malloc(sizeof(double) * B);
  double *r2 = (double *)malloc(sizeof(double) * B);
  double *Nn = (double *)malloc(sizeof(double) * B);
  if (!x || !r2 || !Nn) {
    free(x);
    free(r2);
    free(Nn);
    return -1;
  }
  const double vol = 4.0 * COND_PI * rho_g_cm3 / 3.0;  /* x = vol r^3 */
  for (int k = 0; k < B; ++k) {
    x[k] = cond_grid_mass(x1_g, s_grid, k);
    const double r = cbrt(x[k] / vol);
    r2[k] = r * r;
  }
  for (int64_t pt = 0; pt < npoints; ++pt) {
    double *Np = N + pt * B;
    const double growth = 2.0 * gcoef_cm2_s[pt] * ssat[pt] * dt;
    for (int32_t st = 0; st < nsteps; ++st) {
      if (growth == 0.0) break; /* [R22] s = 0: nothing moves */
      for (int k = 0; k < B; ++k) Nn[k] = 0.0;
      double evap = 0.0;
      for (int k = 0; k < B; ++k) {
        const double n = Np[k];
        if (n == 0.0) continue;
        const double rr = r2[k] + growth;
        if (!(rr > 0.0)) { /* [R24] */
          evap += n * x[k];
          continue;
        }
        const double xn = vol * (rr * sqrt(rr)); /* [R23] */
        if (xn < x[0]) { /* [R24] */
          evap += n * x[k];
          continue;
        }
        if (xn >= x[B - 1]) { /* [R25] */
          Nn[B - 1] += n;
          continue;
        }
        int j = 0;
        while (!(x[j + 1] > xn)) ++j; /* x_j <= xn < x_{j+1} */
        const double phi = (xn - x[j]) / (x[j + 1] - x[j]);
        Nn[j] += n * (1.0 - phi);
        Nn[j + 1] += n * phi;
      }
      for (int k = 0; k < B; ++k) Np[k] = Nn[k];
      if (evaporated) evaporated[pt] += evap;
    }
  }
  free(x);
  free(r2);
  free(Nn);
  return 0;
}
