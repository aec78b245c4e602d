/*
 * fsbm_coal.h -- C ABI of the MI355X (gfx950) collision-coalescence library.
 *
 * The library advances the bin spectra of many independent grid points by
 * the collision-coalescence term of the bin equation (Sec. III, eq. (1)),
 * solved with Bott's flux method (the routine the paper offloads, Sec. III
 * and Sec. VI), with the collection kernels of every pair of particle types
 * tabulated at a few pressure levels and interpolated linearly for each
 * point's pressure (Sec. VI-A, "Lookup optimization"), and with the work
 * restricted to cloudy points (the predicate array of Sec. VI-B).  The
 * same handle also advances the other per-bin process terms of eq. (1) for
 * its spectra: sedimentation in vertical columns (fsbm_coal_sediment), and
 * for the first species (the drops) condensation/evaporation at a given
 * supersaturation (fsbm_coal_condense) and spontaneous breakup
 * (fsbm_coal_set_breakup, fsbm_coal_breakup).
 *
 * All functions return 0 on success or a negative FSBM_E* code; none aborts
 * or throws.  fsbm_coal_strerror() turns a code into text; the handle keeps
 * the message of the last HIP error it saw.
 *
 * Units: N in cm^-3 per bin, bin masses in g, kernels in cm^3 s^-1, pressure
 * in hPa, time in s.
 */
#ifndef FSBM_COAL_H
#define FSBM_COAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define FSBM_OK 0
#define FSBM_EINVAL (-1)       /* bad size, pointer, level order, dt, ... */
#define FSBM_ENOMEM (-2)       /* device or host allocation failed */
#define FSBM_EHIP (-3)         /* HIP runtime error (text kept in handle) */
#define FSBM_EUNSUPPORTED (-4) /* valid but beyond what was compiled */
#define FSBM_EDOMAIN (-5)      /* debug checks: negative, NaN or infinite
                                  input */

/* arithmetic of the pair loop */
#define FSBM_FP64 0  /* every step in FP64 */
#define FSBM_FP32C 1 /* FP32 pair arithmetic (collided masses, flux
                        fraction, transcendentals) on masses normalised by
                        the point's FP64 total; the FP32 amounts are summed
                        per bin in FP64 (each enters exactly, so a transfer
                        leaves and enters with the same value); FP64 final
                        update.  From a point's first step that needs the
                        positivity limiter (or, several species, would
                        drain a bin by more than half), its remaining steps
                        of the call run in FP64.  Two to four species on
                        the doubling grid with 33 bins run one point per
                        lane (points grouped by the species they hold),
                        other shapes one point per wave. */

/* update order of the pairs within a step */
#define FSBM_ORDER_SIMULTANEOUS 0 /* every pair from the step's start state,
                                     per-bin gain and loss sums, positivity
                                     limiter when a bin is over-demanded */
#define FSBM_ORDER_SEQUENTIAL 1   /* Bott's original in-place form: pairs in
                                     order (i ascending, then j >= i), each
                                     seeing the mass the pairs before it
                                     moved; per-pair caps keep every bin
                                     non-negative.  One species on the
                                     doubling grid (s == 1), B in {3, 8, 16,
                                     33, 40}, FSBM_FP64 only */

/* option flags */
#define FSBM_FLAG_DEBUG_CHECKS 1 /* validate N (>= 0, finite) before a step */
#define FSBM_FLAG_NO_GRAPH 2     /* launch kernels directly, no hipGraph */
#define FSBM_FLAG_FORCE_WAVE 4   /* use the one-point-per-wave kernel even
                                    where the one-point-per-lane one fits */
#define FSBM_FLAG_PROFILE 8      /* launch directly (no hipGraph) and time
                                    every collision-kernel launch with HIP
                                    events on the caller's stream; see
                                    fsbm_coal_stats.kernel_ms */

typedef struct fsbm_coal_s *fsbm_coal_t;

typedef struct {
  double x1_g;              /* mass of bin 0; default 3.3510321638291124e-11
                               (a 2 um water drop) */
  int32_t s;                /* bin mass ratio 2^(1/s); default 1 (doubling) */
  const int32_t *product;   /* [S*S] host, product species of a collision of
                               species a and b, symmetric; NULL = default
                               (every collision yields species 0 if S == 1;
                               for S > 1 NULL is an error) */
  int32_t precision;        /* FSBM_FP64 (default) or FSBM_FP32C */
  double theta;             /* bin activity threshold relative to the point's
                               total mass; default 1e-30 */
  int32_t steps_per_launch; /* time steps fused into one kernel launch;
                               0 = choose (tuning cache or default) */
  int32_t flags;            /* FSBM_FLAG_* */
  int32_t order;            /* FSBM_ORDER_SIMULTANEOUS (default) or
                               FSBM_ORDER_SEQUENTIAL; a sequential handle
                               outside the shapes above is FSBM_EUNSUPPORTED
                               at create */
} fsbm_coal_opts;

/* Fill opts with the defaults above. */
void fsbm_coal_opts_default(fsbm_coal_opts *opts);

/*
 * Create a handle for one bin grid and species set (Sec. VI-A: collection
 * kernels per particle-type pair at pressure levels).
 *  nbins          B >= 2 bins per species (mass grid x_k = x1 2^(k/s))
 *  nspecies       S in [1, 8]
 *  kernel_tables  host, FP64, [S(S+1)/2][L][B][B]; species pairs in the order
 *                 (0,0),(0,1),..,(0,S-1),(1,1),..; for pair (a,b) entry
 *                 [l][i][j] is the kernel of species a bin i with species b
 *                 bin j at level l.  Copied; the caller keeps ownership.
 *  nlevels        L >= 1
 *  p_levels_hpa   host, [L], strictly decreasing (e.g. 1000, 750, 500)
 *  opts           NULL for defaults
 *  out            receives the handle
 * Errors: FSBM_EINVAL (sizes, levels, product map, non-finite or negative
 * table entries), FSBM_EUNSUPPORTED (B > 512, more than 8 pressure brackets,
 * or S*B > 768 where the one-point-per-lane kernels do not apply; checked
 * before any device call), FSBM_ENOMEM, FSBM_EHIP.  Uses the current HIP
 * device.
 */
int fsbm_coal_create(int32_t nbins, int32_t nspecies,
                     const double *kernel_tables, int32_t nlevels,
                     const double *p_levels_hpa, const fsbm_coal_opts *opts,
                     fsbm_coal_t *out);

/*
 * Advance npoints grid points by nsteps collision steps of dt_s seconds
 * (Sec. VI-B: the offloaded collision loop over all points whose predicate
 * holds; here a point takes part iff it holds mass).
 *  N       device, FP64, C-contiguous [npoints][S][B], updated in place
 *  p_hpa   device, FP64, [npoints] pressure of each point
 *  stream  a hipStream_t (NULL = the default stream)
 * Stream-ordered and asynchronous: returns once the work is enqueued.  Launch
 * and argument errors are returned; device faults surface at the caller's
 * next synchronisation.  npoints == 0 or nsteps == 0 is a no-op.  The caller
 * owns N and p and keeps them alive until the stream has passed the step.
 * One step may be in flight per handle (the handle owns the workspace).
 */
int fsbm_coal_step(fsbm_coal_t h, double *N, const double *p_hpa,
                   int64_t npoints, double dt_s, int32_t nsteps,
                   void *stream);

/*
 * fsbm_coal_step with the temperature gates of FSBM's loop over grid points
 * (Sec. III, main-loop listing): a point's microphysics runs only where its
 * previous temperature exceeds 193.15 K, and the collision routine within it
 * only where the current temperature exceeds 223.15 K.  A point takes part
 * in the call iff it holds mass, t_old_k[pt] > 193.15 and
 * t_now_k[pt] > 223.15 (strict; a NaN temperature fails); every other point
 * is left unchanged bit for bit, and fsbm_coal_totals reports its mass and
 * number as both before and after.
 *  t_old_k  device, FP64, [npoints] previous temperature (K), or NULL (that
 *           test passes for every point)
 *  t_now_k  device, FP64, [npoints] current temperature (K), or NULL
 * Other arguments, ownership, errors and results (for the points that pass)
 * as fsbm_coal_step, which is this call with both arrays NULL.  The
 * temperatures are read on the device when the call runs, like N.
 */
int fsbm_coal_step_gated(fsbm_coal_t h, double *N, const double *p_hpa,
                         const double *t_old_k, const double *t_now_k,
                         int64_t npoints, double dt_s, int32_t nsteps,
                         void *stream);

/*
 * fsbm_coal_step without any device allocation, for callers that cannot
 * allocate: code running under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results (bit for bit),
 * ownership and errors as fsbm_coal_step, except:
 *  - the call's workspace is a fixed block of 64 MiB (67108864 bytes) of
 *    static device memory in the library, one per GPU, held from the
 *    library's first use on that GPU until the process ends.  A call whose
 *    workspace does not fit returns FSBM_EUNSUPPORTED before enqueueing
 *    anything (fsbm_coal_last_error gives the bytes needed).  The workspace
 *    takes about 2 S B 8 + 54 bytes per point on the one-point-per-lane
 *    kernels (one species on the doubling grid, B <= 40) and S B 8 + 50
 *    bytes per point otherwise: about 110,000 points at 33 bins and one
 *    species, 60,000 at four species;
 *  - the call enqueues kernels only: no allocation, no hipGraph of its own,
 *    no host synchronisation, so it may itself be captured into a caller's
 *    graph.  FSBM_FLAG_DEBUG_CHECKS and FSBM_FLAG_PROFILE are ignored;
 *  - every call on one GPU, from any handle, shares that GPU's block and
 *    overwrites it: calls that overlap in time on one GPU (different streams
 *    or threads) race and give undefined results; serialise them.
 *    fsbm_coal_totals and fsbm_coal_get_stats after such a call read the
 *    block, so they hold only until the next call of this entry point on
 *    that GPU.
 * Also FSBM_EHIP if the block's device address could not be obtained.
 */
int fsbm_coal_step_noalloc(fsbm_coal_t h, double *N, const double *p_hpa,
                           int64_t npoints, double dt_s, int32_t nsteps,
                           void *stream);

/*
 * One launch sequence over several handles with different grids (mixed
 * 33/66/132-bin batches): the cloudy points of every grid are compacted into
 * one work list and advanced by one persistent kernel per group of fused
 * steps.  Arrays are indexed by grid; same ownership rules as
 * fsbm_coal_step.  All handles must use the same precision and device, be
 * distinct, have S*B <= 768 and the simultaneous order; at most 4 grids.  Results equal those of
 * fsbm_coal_step per grid with the one-point-per-wave kernel, bit for bit.
 * The pair, limiter and exact-path counters and the profiled launch
 * timings of the call are kept in the handle with the largest S*B (the
 * first one listed if several tie); active_points stays per handle.
 */
int fsbm_coal_step_multi(const fsbm_coal_t *hs, int32_t ngrids,
                         double *const *N, const double *const *p_hpa,
                         const int64_t *npoints, double dt_s, int32_t nsteps,
                         void *stream);

/*
 * Sedimentation of the handle's S x B bin spectra in vertical columns: the
 * term d((w - V_t) f)/dz of the bin equation (Sec. III, eq. (1)) in still
 * air (w = 0), first-order upwind in flux form, explicit.  Per (column,
 * species-bin) each step of dt_s seconds is taken in n equal sub-steps,
 * n = max(1, ceil(max over levels of v_l dt_s / dz_l)); per sub-step tau,
 * with the values at its start and levels numbered from the bottom,
 * F_l = v_l N_l tau leaves level l through its bottom face,
 * N_l += (F_{l+1} - F_l) / dz_l (nothing enters the top level), and F_0 is
 * added to the column's precipitation.  Number is conserved (column
 * content plus precipitation) and N stays >= 0.
 *  N           device, FP64, [npoints][S][B], updated in place; point
 *              (column c, level l) is c * col_stride + l * lev_stride
 *              (column-major grids: col_stride = nlev, lev_stride = 1;
 *              [nz][ny][nx] grids: 1 and nx * ny).  Every addressed point
 *              must lie in the caller's array.
 *  ncols, nlev columns and levels, 1 <= nlev <= 64 (level 0 at the bottom)
 *  dz_cm       device, FP64, [nlev] layer thickness (cm), > 0
 *  v_cm_s      device, FP64, [S][B] fall speed (cm/s), >= 0
 *  vfac        device, FP64, [ncols][nlev] factor on the fall speed at
 *              each column and level (air-density correction), or NULL (1)
 *  precip      device, FP64, [ncols][S][B], number per cm^2 that left the
 *              bottom level, added to; or NULL
 * Stream-ordered and asynchronous; ncols == 0 or nsteps == 0 is a no-op.
 * Errors: FSBM_EINVAL (sizes, strides, dt, null pointers),
 * FSBM_EUNSUPPORTED (nlev > 64), FSBM_EHIP.  dz_cm and v_cm_s are read on
 * the device: values outside the ranges above give undefined results.
 */
int fsbm_coal_sediment(fsbm_coal_t h, double *N, int64_t ncols, int32_t nlev,
                  int64_t col_stride, int64_t lev_stride, const double *dz_cm,
                  const double *v_cm_s, const double *vfac, double dt_s,
                  int32_t nsteps, double *precip, void *stream);

/*
 * Condensation and evaporation of the first species' spectrum (liquid
 * water drops, density 1 g/cm^3) at a prescribed supersaturation: the
 * condensation term of the bin equation (Sec. III, eq. (1)), the process
 * the paper names as the next to offload (Sec. VIII).  Per point and step
 * of dt_s seconds, every drop of bin k (radius r_k of the sphere of mass
 * x_k) grows by r dr/dt = G s, i.e. r^2 -> r_k^2 + 2 G s dt_s, to the mass
 * x' = (4 pi / 3) (r_k^2 + 2 G s dt_s)^(3/2).  Its number goes to the grid
 * bins j, j+1 with x_j <= x' < x_{j+1} as N (1 - phi) and N phi,
 * phi = (x' - x_j) / (x_{j+1} - x_j), which keeps number and mass;
 * contributions are summed in ascending source bin.  Drops with
 * r_k^2 + 2 G s dt_s <= 0 or x' < x_0 evaporate (their mass N x_k is added
 * to evaporated); drops with x' >= x_{B-1} stay in the last bin.  Other
 * species are not touched.  The vapour and heat budgets (the feedback on s
 * and G) are the caller's.  The result equals this definition bit for bit
 * (FP64, correctly rounded square root and division).
 *  N           device, FP64, [npoints][S][B], bins of species 0 updated in
 *              place
 *  ssat        device, FP64, [npoints] supersaturation over water as a
 *              fraction (s < 0 evaporates)
 *  gcoef_cm2_s device, FP64, [npoints] growth coefficient G (cm^2/s)
 *  evaporated  device, FP64, [npoints] evaporated mass (g/cm^3), added to
 *              once per step; or NULL
 * Points whose species-0 bins are all zero, or whose 2 G s dt_s is zero,
 * are left as they are (evaporated included).  Stream-ordered and
 * asynchronous; npoints == 0 or nsteps == 0 is a no-op.  The first call,
 * and a call with more points than any before, allocates the handle's
 * condensation workspace (synchronous); calls on one handle must not
 * overlap.  Errors: FSBM_EINVAL (sizes, dt, null pointers),
 * FSBM_EUNSUPPORTED (npoints >= 2^31), FSBM_ENOMEM, FSBM_EHIP.  Any grid of
 * the library's (B <= 512 bins per species) is supported: 33 and 66 bins
 * run one point per lane, larger grids one point per wave.
 */
int fsbm_coal_condense(fsbm_coal_t h, double *N, int64_t npoints,
                       const double *ssat, const double *gcoef_cm2_s,
                       double dt_s, int32_t nsteps, double *evaporated,
                       void *stream);

/*
 * Breakup tables of the first species for fsbm_coal_breakup: the breakup
 * term of the bin equation (Sec. III, eq. (1)) in the linear form of
 * spontaneous breakup (Srivastava 1971): a drop of bin l breaks at the rate
 * rate_per_s[l] (s^-1) into fragments[l * B + k] drops of each smaller bin
 * k < l; the caller balances the table's mass,
 * sum_k fragments[l * B + k] x_k = x_l (mass is kept to that balance).
 *  rate_per_s  host, FP64, [B], finite and >= 0; bin 0's is ignored (the
 *              smallest drops do not break)
 *  fragments   host, FP64, [B][B], finite and >= 0, zero for k >= l
 * Both are copied; the caller keeps them.  The device copy is made by the
 * next fsbm_coal_breakup.  Errors: FSBM_EINVAL (null, negative or
 * non-finite entries, fragments on or above the diagonal).  Any grid of
 * the library's (B <= 512 bins per species) is supported.
 */
int fsbm_coal_set_breakup(fsbm_coal_t h, const double *rate_per_s,
                          const double *fragments);

/*
 * Spontaneous breakup of the first species' spectrum with the tables of
 * fsbm_coal_set_breakup.  Per point and step of dt_s seconds, the share
 * b_l = 1 - exp(-P_l dt_s) of bin l's drops breaks (fragments do not break
 * again within the step):
 *   N'_k = (N_k - b_k N_k) + sum_{l>k} (b_l N_l) fragments[l][k],
 * summed in ascending l.  Other species are not touched.  The result
 * equals this definition bit for bit (FP64, b computed on the host with
 * expm1).
 *  N           device, FP64, [npoints][S][B], bins of species 0 updated in
 *              place
 * Points without drops in bins 1..B-1 are left as they are.
 * Stream-ordered and asynchronous; npoints == 0 or nsteps == 0 is a no-op.
 * The first call, a call with more points than any before, and a call with
 * a dt_s other than the previous call's (or after new tables) synchronise
 * the device and upload b and the table; calls on one handle must not
 * overlap.  Errors: FSBM_EINVAL (sizes, dt, null N, no tables set),
 * FSBM_EUNSUPPORTED (npoints >= 2^31), FSBM_ENOMEM, FSBM_EHIP.  33 and 66
 * bins run one point per lane, larger grids one point per wave.
 */
int fsbm_coal_breakup(fsbm_coal_t h, double *N, int64_t npoints, double dt_s,
                      int32_t nsteps, void *stream);

/*
 * Explicitly autotune the kernel family and launch shape for about
 * npoints_hint cloudy points, timing candidates on synthetic states.
 * Candidates: steps per launch and waves per block (one point per lane);
 * where the several-species lane kernels apply (FP32C, two to four species,
 * doubling grid, 33 bins), those and the one-point-per-wave kernel, each
 * with steps per launch (and persistent blocks); the fastest one that
 * passes the checks is kept.  Within a family every candidate must repeat
 * the family's first result bit for bit; a second family must agree with
 * the first within 2e-5 of each bin's mass (fsbm_coal_stats counts
 * candidates run and rejected).
 * Synchronises the stream.  The choice is kept in the handle and in the
 * cache file named by the FSBM_TUNE_CACHE environment variable, if set.
 * The synthetic runs use the handle's workspace: until the next step,
 * fsbm_coal_totals returns FSBM_EINVAL and fsbm_coal_get_stats reports no
 * counters of a step call.  Errors: FSBM_EINVAL, FSBM_EHIP (allocation or
 * runtime failure; nothing is leaked).
 */
int fsbm_coal_tune(fsbm_coal_t h, int64_t npoints_hint, void *stream);

/*
 * Per-point FP64 bookkeeping of the last fsbm_coal_step on this handle:
 * total mass (g cm^-3) and number (cm^-3) of each point before the first and
 * after the last step.  Each pointer is device [npoints] or NULL.  Enqueued
 * on the stream of that step.
 */
int fsbm_coal_totals(fsbm_coal_t h, double *mass_before, double *mass_after,
                     double *num_before, double *num_after);

typedef struct {
  int64_t active_points;  /* cloudy points in the last step call */
  int64_t pair_evals;     /* bin pairs evaluated (both bins active, merged
                             mass inside the grid, kernel entry nonzero at
                             some tabulated level), summed over points and
                             steps of the last call */
  int64_t limiter_steps;  /* point-steps where the positivity limiter ran;
                             sequential order: pairs at which a positivity
                             cap applied */
  int64_t fp64_fallback_steps; /* point-steps taken in FP64 outside the
                                  fast path: one point per lane, once the
                                  fast kernel finds that the limiter may
                                  fire, the point takes every remaining step
                                  of the call on the exact FP64 path; one
                                  point per wave in FP32C mode, once the
                                  limiter fires the point takes that and
                                  every remaining step of the call in FP64
                                  mode */
  int32_t kernel;         /* kernel family of the last call (before any
                             call: the one a call would use): 0 = one
                             point per lane, 1 = one point per wave, 2 =
                             one point per lane, sequential, 3 = one point
                             per lane for two to four species (FP32C) */
  int32_t steps_per_launch;
  int32_t waves_per_block;
  int32_t kernel_launches; /* FSBM_FLAG_PROFILE: collision-kernel launches
                              timed since the handle was created */
  double kernel_ms;        /* FSBM_FLAG_PROFILE: their summed duration */
  int64_t exact_pair_evals; /* the part of pair_evals evaluated on the
                               exact FP64 path of points that left the fast
                               kernel (see fp64_fallback_steps) */
  int64_t graph_captures;  /* hipGraphs this handle has captured since it
                              was created: a call replays the handle's
                              cached graph only while the call's
                              arguments, launch shape and the workspaces
                              of every handle in it are unchanged */
  int32_t tune_candidates; /* the last fsbm_coal_tune: candidates run */
  int32_t tune_rejected;   /* ... and rejected: a launch shape whose result
                              differs from its family's first candidate by
                              a bit, or a kernel family whose result
                              differs from the first family's by more than
                              2e-5 of a bin's mass (floor 1e-9 of the
                              point's mass) */
} fsbm_coal_stats;

/* Counters of the last step call.  Synchronises that call's stream. */
int fsbm_coal_get_stats(fsbm_coal_t h, fsbm_coal_stats *out);

/* Free every resource of the handle; NULL is accepted.  Using a handle after
   destroy is undefined. */
int fsbm_coal_destroy(fsbm_coal_t h);

/* Static text for an error code. */
const char *fsbm_coal_strerror(int code);

/* Message of the last HIP error seen by the handle ("" if none). */
const char *fsbm_coal_last_error(fsbm_coal_t h);

#ifdef __cplusplus
}
#endif
#endif
