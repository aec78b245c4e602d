/*
 * fsbm_oracle_sed.c -- plain FP64 CPU oracle of the sedimentation term of
 * the bin equation.  TEST INFRASTRUCTURE ONLY (see fsbm_oracle.h): loaded by
 * the tests, the smoke check and the benchmark's CPU-baseline leg, never by
 * the GPU library; it shares no code with it.
 *
 * Sec. III, eq. (1): the number density f of bin k of particle type i moves
 * vertically with w - V_t, V_t the bin's terminal fall speed; this is the
 * term d((w - V_t) f)/dz.  The paper gives no discretisation.  Readings
 * taken here ([R18]-[R21]):
 *  [R18] still air (w = 0): the vertical air motion is the dynamics' part of
 *        eq. (1); sedimentation moves each bin down with its own V_t >= 0;
 *  [R19] first-order upwind flux form, explicit in time: with levels
 *        numbered from the bottom, layer thickness dz_l and fall speed v_l,
 *        the number per unit area leaving level l through its bottom face
 *        during a (sub-)step tau is F_l = v_l N_l tau, from the values at
 *        the start of the sub-step; then N_l' = N_l + (F_{l+1} - F_l) / dz_l
 *        with F_{nlev} = 0 (nothing enters the top level), and F_0, what
 *        leaves the bottom level, is the precipitation, accumulated per
 *        column, species and bin (cm^-2);
 *  [R20] each step dt of each (column, species, bin) is taken in n equal
 *        sub-steps tau = dt / n, n = max(1, ceil(max over levels of
 *        v_l dt / dz_l)), so that no level passes on more than it holds;
 *  [R21] v_l = V(s, k) * vfac_l: a fall speed per species and bin at a
 *        reference state times a factor per column and level (the
 *        air-density correction; 1 where none is given).
 * The scheme conserves number exactly up to rounding (what leaves a level
 * enters the next one or the precipitation), keeps N >= 0 for Courant
 * numbers <= 1 and moves the first vertical moment of a profile down at
 * exactly v per unit time while nothing reaches the ground; with a uniform
 * Courant number C a single-level pulse spreads as the binomial
 * distribution of n trials with probability C.  The tests pin these.
 *
 * Layout: point (column c, level l) is point c * col_stride + l * lev_stride
 * of N [npoints][S][B], so that both column-major and level-major grids
 * (e.g. [nz][ny][nx]) can be used in place; dz_cm is [nlev], v_cm_s [S][B],
 * vfac [ncols][nlev] (or NULL), precip [ncols][S][B] (or NULL; added to).
 */
#include "fsbm_oracle.h"

#include <math.h>
#include <stdlib.h>

int fsbm_oracle_sediment(int32_t nspecies, int32_t nbins, int64_t ncols,
                         int32_t nlev, int64_t col_stride,
                         int64_t lev_stride, double *N, const double *dz_cm,
                         const double *v_cm_s, const double *vfac,
                         double dt, int32_t nsteps, double *precip) {
  if (nspecies < 1 || nbins < 1 || ncols < 0 || nlev < 1 || nsteps < 0 ||
      !(dt > 0.0) || !isfinite(dt) || !N || !dz_cm || !v_cm_s)
    return -1;
  for (int32_t l = 0; l < nlev; ++l)
    if (!(dz_cm[l] > 0.0) || !isfinite(dz_cm[l])) return -1;
  const int64_t SB = (int64_t)nspecies * nbins;
  for (int64_t q = 0; q < SB; ++q)
    if (!(v_cm_s[q] >= 0.0) || !isfinite(v_cm_s[q])) return -1;
  double *F = (double *)malloc(sizeof(double) * (size_t)nlev);
  if (!F) return -1;
  for (int64_t c = 0; c < ncols; ++c) {
    for (int64_t q = 0; q < SB; ++q) {
      /* [R20] sub-steps of this column, species and bin */
      double cmax = 0.0;
      for (int32_t l = 0; l < nlev; ++l) {
        const double fac = vfac ? vfac[c * nlev + l] : 1.0;
        const double cl = v_cm_s[q] * fac * dt / dz_cm[l];
        if (cl > cmax) cmax = cl;
      }
      int64_t nsub = (int64_t)ceil(cmax);
      if (nsub < 1) nsub = 1;
      const double tau = dt / (double)nsub;
      for (int32_t st = 0; st < nsteps; ++st)
        for (int64_t u = 0; u < nsub; ++u) {
          /* [R19] fluxes from the old values, then the update */
          for (int32_t l = 0; l < nlev; ++l) {
            const double fac = vfac ? vfac[c * nlev + l] : 1.0;
            const double Nl = N[(c * col_stride + l * lev_stride) * SB + q];
            F[l] = v_cm_s[q] * fac * Nl * tau;
          }
          for (int32_t l = 0; l < nlev; ++l) {
            const double in = (l + 1 < nlev) ? F[l + 1] : 0.0;
            double *Nl = &N[(c * col_stride + l * lev_stride) * SB + q];
            *Nl = *Nl + (in - F[l]) / dz_cm[l];
          }
          if (precip) precip[c * SB + q] += F[0];
        }
    }
  }
  free(F);
  return 0;
}
