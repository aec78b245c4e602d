/*
 * fsbm_oracle.h -- plain FP64 CPU oracle of the FSBM collision-coalescence
 * step (stochastic collection equation, Bott-style flux redistribution).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with
 * the GPU library and the GPU library never calls it.
 *
 * What it computes (per grid point, per time step; the paper names the
 * routine as Bott's flux method for the collision term of the bin equation,
 * Sec. III eq. (1), and describes per-point pressure-interpolated kernel
 * tables, Sec. VI-A "Lookup optimization"):
 *   S1  M = N*x, M_tot (species then bins, ascending); M_tot == 0 -> unchanged
 *   S2  bin active iff M >= theta*M_tot
 *   S3  K(p) piecewise-linear between tabulated pressure levels, clamped
 *   S4  canonical pair loop, Bott exponential-profile flux fraction
 *   S5  positivity limiter (only when some bin is over-demanded)
 *   S6  M' = M + (G - L), negative round-off clamped to 0, N' = M'/x
 *   S7  per-point mass / number before and after the call
 * Every arithmetic choice the paper leaves open is a reading, marked [R#]
 * where it shapes the arithmetic in fsbm_oracle.c.
 *
 * Units: N in cm^-3 per bin, x in g, K in cm^3 s^-1, p in hPa, dt in s.
 */
#ifndef FSBM_ORACLE_H
#define FSBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nbins;            /* B >= 2 */
  int32_t nspecies;         /* S in [1, 8] */
  int32_t nlevels;          /* L >= 1 */
  int32_t s;                /* bin mass ratio 2^(1/s), s >= 1 */
  double x1_g;              /* mass of bin 0 in g */
  double theta;             /* activity threshold relative to M_tot */
  const double *tables;     /* [S(S+1)/2][L][B][B]; pair (a,b), a<=b, entry
                               [i][j] = species a bin i with species b bin j */
  const double *p_levels;   /* [L], hPa, strictly decreasing */
  const int32_t *product;   /* [S*S] product species of (a,b), symmetric */
  int32_t order;            /* 0 = simultaneous update of every pair from
                               the step's start state (S1-S6);
                               1 = Bott's sequential in-place update, one
                               species only (no limiter: a per-pair cap) */
} fsbm_oracle_desc;

/* Advance npoints independent points by nsteps steps of dt, in place.
 * N: host [npoints][S][B].  p: host [npoints].  Optional outputs (may be
 * NULL): per-point total mass / number before the first and after the last
 * step, the number of point-steps in which the limiter fired, per point
 * the number of its steps in which it fired, and per point and bin
 * ([npoints][S][B] bytes) 1 where the limiter scaled that bin's demand at
 * some step of the call (sigma < 1), else 0.  With order == 1 the counts
 * are of capped pairs instead (summed over all pairs and steps) and the
 * bins marked are those a cap left empty.
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad input. */
int fsbm_oracle_run(const fsbm_oracle_desc *d, double *N, const double *p,
                    int64_t npoints, double dt, int32_t nsteps,
                    double *mass_before, double *mass_after,
                    double *num_before, double *num_after,
                    int64_t *limiter_steps, int32_t *limiter_per_point,
                    unsigned char *limited_bins, int32_t nthreads);

/* The same, for the points whose collision call the main loop makes
 * (Sec. III listing): a point is advanced only if t_old[pt] > 193.15 K and
 * t_now[pt] > 223.15 K (K; either array NULL = that test passes); the
 * other points are left unchanged. */
int fsbm_oracle_run_gated(const fsbm_oracle_desc *d, double *N,
                          const double *p, const double *t_old,
                          const double *t_now, int64_t npoints, double dt,
                          int32_t nsteps, double *mass_before,
                          double *mass_after, double *num_before,
                          double *num_after, int64_t *limiter_steps,
                          int32_t *limiter_per_point,
                          unsigned char *limited_bins, int32_t nthreads);

/* Bin masses x_k, k = 0..B-1. */
int fsbm_oracle_grid(const fsbm_oracle_desc *d, double *x);

/* Target bin k_ij and Courant number c_ij for every bin pair, [B][B].
 * k = -1 marks a pair whose merged mass leaves the grid. */
int fsbm_oracle_targets(const fsbm_oracle_desc *d, int32_t *k, double *c);

/* Flux fraction f(c, x1) after the clamp to [0, 1]. */
double fsbm_oracle_flux_fraction(double c, double x1);

/* Interpolated kernel entry K^{ab}_{ij}(p). */
double fsbm_oracle_kernel_at(const fsbm_oracle_desc *d, double p, int32_t a,
                             int32_t b, int32_t i, int32_t j);

/* Number of threads OpenMP would use. */
int fsbm_oracle_max_threads(void);

/* Sedimentation of columns: the term d((w - V_t) f)/dz of eq. (1) (Sec. III)
 * in still air, first-order upwind in flux form, explicit, each step split
 * into equal sub-steps with Courant numbers <= 1 (readings R18-R21, see
 * fsbm_oracle_sed.c).  N: host [npoints][S][B], in place; point (column c,
 * level l, level 0 at the bottom) is c * col_stride + l * lev_stride.
 * dz_cm [nlev] > 0; v_cm_s [S][B] >= 0; vfac [ncols][nlev] or NULL;
 * precip [ncols][S][B] or NULL, the number per cm^2 leaving the bottom level
 * is added to it.  Returns 0, or -1 on bad input. */
int fsbm_oracle_sediment(int32_t nspecies, int32_t nbins, int64_t ncols,
                         int32_t nlev, int64_t col_stride,
                         int64_t lev_stride, double *N, const double *dz_cm,
                         const double *v_cm_s, const double *vfac,
                         double dt, int32_t nsteps, double *precip);

/* Condensation/evaporation of one species' spectrum at a prescribed
 * supersaturation (fsbm_oracle_cond.c, readings R22-R25): N [npoints][nbins]
 * updated in place over nsteps steps of dt; ssat, gcoef_cm2_s [npoints];
 * evaporated [npoints] (g/cm^3) added to once per step, or NULL.  Grid
 * x_k = x1 2^(k/s_grid) (exact doubling); spheres of density rho.  Returns
 * 0, or -1 on bad input. */
int fsbm_oracle_condense(int32_t nbins, int32_t s_grid, double x1_g,
                         double rho_g_cm3, int64_t npoints, double *N,
                         const double *ssat, const double *gcoef_cm2_s,
                         double dt, int32_t nsteps, double *evaporated);

/* Spontaneous breakup of one species' spectrum (fsbm_oracle_break.c,
 * readings R26-R28): N [npoints][nbins] updated in place over nsteps steps
 * of dt; rate_per_s [nbins] >= 0 (bin 0's is ignored); fragments
 * [nbins][nbins] >= 0, row l the fragments per broken drop of bin l, zero
 * on and above the diagonal.  Returns 0, or -1 on bad input. */
int fsbm_oracle_breakup(int32_t nbins, int64_t npoints, double *N,
                        const double *rate_per_s, const double *fragments,
                        double dt, int32_t nsteps);

#ifdef __cplusplus
}
#endif
#endif
