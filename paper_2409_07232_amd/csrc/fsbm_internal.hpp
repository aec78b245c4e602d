// fsbm_internal.hpp -- structures shared by the host library and the
// gfx950 kernels of the collision-coalescence step.  Internal: not part of
// the C ABI (include/fsbm_coal.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsbm {

// ln 2 in FP32, shared by the host tables and the kernels
constexpr float kLn2f = 0.69314718055994530942f;


constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxSpecies = 8;
constexpr int kMaxBins = 512;
constexpr int kMaxBrackets = 8;    // pressure brackets (levels - 1), capped
// compaction buckets: pressure brackets, or (multi-species lane kernels)
// pairs of a bracket and a species set
constexpr int kMaxBuckets = 64;
constexpr int kLaneMaxBins = 40;   // one-point-per-lane kernel: S*B limit
constexpr int kSlotAlign = 256;    // slot capacity granularity (>= block)
constexpr int kMaxOwn = 12;        // one-point-per-wave kernel: bins per lane
constexpr int kOwnSmall = 4;       // its builds for grids of fewer bins
constexpr int kOwnMid = 8;         //   per lane
constexpr int kMaxGrids = 4;       // grids in one multi-grid launch
// one-point-per-lane kernels for several species: species and S*B limits
constexpr int kMultiMaxSpecies = 4;
constexpr int kMultiMaxSB = 132;
constexpr int kNumCounters = 5;    // device counters of a step call
// Empty-neighbour guard of the flux fraction: x1 >= ln(1e-60).
constexpr double kX1Floor = -138.15510557964274;

// Read-only description of one bin grid and species set, device pointers.
struct DevModel {
  int B, S, L, s;
  int nbr;        // pressure brackets = max(L - 1, 1)
  int nmask;      // compaction buckets per bracket: 1, or 2^S where the
                  // multi-species lane kernels bucket points by species set
  int npairs;     // S (S + 1) / 2 species pairs
  unsigned bmagic;  // ceil(2^32 / B): q / B = umulhi(q, bmagic) for q < 2^32 / B
  double theta;
  const double *x;      // [B] bin masses (g)
  const float *xf;      // [B] bin masses rounded to FP32
  const double *invx;   // [B] 1 / x
  const float *invxf;   // [B] 1 / x rounded to FP32
  const int *kt;        // [B*B] target bin of pair (i, j), -1 = off grid
  const double *ct;     // [B*B] Courant number c_ij (FP64)
  const float *ctf;     // [B*B] c_ij rounded to FP32
  const int *product;   // [S*S] product species
  const double *Kd;     // [npairs][nbr][B][B][2] (K_{l+1}, K_l - K_{l+1})
  const float *Kf;      // same, FP32
  const double *plev;   // [L]
  // species pair 0 tables transposed to [nbr][j][i][2] and [j][i]: row j of
  // the pair loop reads its columns i < j contiguously
  const double *KdT;
  const float *KfT;
  const double *ctT;
  const float *ctfT;  // [j][i][2]: FP32 Courant number c and 2 (c * kLn2f)
  // species pair 0, row j: bit i (i <= j) set iff the kernel entry [i][j]
  // is nonzero at some tabulated level; a pair whose entry is zero at every
  // level collides nothing (C = 0) and is neither evaluated nor counted
  const unsigned long long *nzT;  // [B]
  // ordered species pairs (a at the smaller bin i, b at the larger bin j),
  // index a * S + b: kernel entries transposed to [nbr][j][i][2] (FP32,
  // multi-species lane kernels only) and, for B <= 64, bit i of row j set
  // iff the entry is nonzero at some level
  const float *KfO;
  const unsigned long long *nzO;  // [S * S][B]
  // [2^S]: the species set a point can hold during a call, from the set it
  // holds (closed under the product map)
  const unsigned char *closure;
  // one-point-per-wave kernel: bins of each lane's per-bin work ([64]
  // [kMaxOwn], -1 padded) and two streams of pair entries, gain entries
  // (grouped by the bin the pair lands in) and loss entries (grouped by the
  // bin that loses mass), each entry holding the pair's static data.  Per
  // species pair (a <= b) and side, the entries in bin order are cut into
  // 64 contiguous equal segments, one per lane, interleaved by lane (entry
  // r of lane l at r * 64 + l); gain blocks first (wrows_g rows), then loss
  // blocks (wrows_l).  A bin whose entries span several lanes is shared
  // (kWShared) and is summed by a fix-up after its block (wfix).
  const short *own;
  int wown;               // bins a lane owns at most (<= kMaxOwn)
  int wrows_g, wrows_l;
  const int *wblk;        // [npairs][4]: gain block row, rows; loss same
  const int *wfixb;       // [npairs][4]: gain fix-up offset, count; loss
  const uint2 *wfix;      // .x = bin | first lane << 16; .y = last lane |
                          // slot of the bin in the first lane << 16
  const uint2 *we_idx;    // .x = qa | qb << 16, .y = q_target | flags << 16
  const float2 *we_x32;   // (x_i, x_j) FP32
  const double2 *we_x64;  // (x_i, x_j)
  const float2 *we_c32;   // (c, 2 c ln 2) FP32
  const double *we_c64;   // c
  const float2 *we_k32;   // [nbr][rows * 64] (K_{l+1}, K_l - K_{l+1}) FP32
  const double2 *we_k64;  // same, FP64
};

// Flags of a wave-stream entry for the pair (a,i) x (b,j), qa = a B + i,
// qb = b B + j, merged mass landing in q_target.
constexpr unsigned kWValid = 1u;  // a pair (not padding)
constexpr unsigned kWTA = 2u;     // qa is the target bin
constexpr unsigned kWTB = 4u;     // qb is the target bin
constexpr unsigned kWSelf = 8u;   // qa == qb (same species and bin)
constexpr unsigned kWSideB = 16u; // loss entry: the owner is qb (else qa)
constexpr unsigned kWFlux = 32u;  // the target is not the top bin: flux
constexpr unsigned kWShared = 64u; // the entry's bin spans several lanes

// Compaction results, written on the device (graph-capturable: no host
// round trip).  Slots of one pressure bracket are contiguous and padded to a
// multiple of the wave size so that every wave shares one bracket.
struct CompactMeta {
  int nslots;                       // total slots incl. padding
  int nactive;                      // cloudy points
  int bucket_base[kMaxBuckets + 1]; // first slot of each bracket, + end
  int bucket_count[kMaxBuckets];    // cloudy points per bracket
};

// Element (q, slot) of the tiled structure-of-arrays state: each wave's 64
// slots form one tile in which bin q of all 64 points is a contiguous
// 512-byte row.
__host__ __device__ __forceinline__ size_t state_index(int q, int slot,
                                                       int SB) {
  return ((size_t)(slot >> 6) * SB + q) * 64 + (slot & 63);
}
// The one-point-per-wave kernel keeps each point's bins contiguous instead.
__host__ __device__ __forceinline__ size_t state_index_aos(int q, int slot,
                                                           int SB) {
  return (size_t)slot * SB + q;
}

// Per-call device workspace of one handle.
struct DevWork {
  int64_t npoints;
  int slot_cap;          // capacity of the slot arrays (stride of state)
  int nblocks;           // compaction blocks (rows of block_counts)
  int *slot_point;       // [slot_cap] point index or -1 (padding)
  double *state;         // tiled SoA [slot/64][S*B][slot%64] bin numbers N
  double *state_alt;     // same shape: second buffer of the lane kernels
  double *wgt;           // [slot_cap] pressure-interpolation weight
  CompactMeta *meta;     // device
  int *block_counts;     // [nblocks_compact][kMaxBuckets]
  int *block_offsets;    // same shape, exclusive scan
  double *tot;           // [4][npoints]: mass before/after, number b/a
  unsigned *keys;        // [slot_cap] sort keys (lane kernels) or null
  int *pending;          // [slot_cap] steps of the call left for the exact
                         // FP64 path (0 = point still on the fast path)
  unsigned char *cloudy;  // [npoints] 1: takes part in the call (holds mass,
                          // passes the temperature gates); 2: holds mass,
                          // gated; 0: no mass
  unsigned long long *counters;  // [kNumCounters]: pair evals, limiter,
                                 // fallback steps, work-queue position of
                                 // the wave kernel, pair evals of the exact
                                 // FP64 path (also in the first)
};

// One grid of a one-point-per-wave launch (a call may cover several grids).
struct WaveGrid {
  DevModel m;
  const int *slot_point;
  double *state;  // [slot][S*B]
  const double *wgt;
  const CompactMeta *meta;
  int *pending;
  int slot_cap;
  int tiled;      // state in the tiled layout of the one-point-per-lane
                  // kernels (the FP64 follow-up of the multi-species ones)
};

struct WaveArgs {
  WaveGrid g[kMaxGrids];
  int ngrids;
  unsigned long long *counters;
  double dt;
  int nsteps;       // steps in this launch
  int steps_left;   // steps of the call left when this launch starts
  int pending_only; // FP64 steps for the points marked pending only
  int launch_idx;   // launches of this call before this one (work queue)
};

// Arguments of the step kernels.
struct StepArgs {
  DevModel m;
  int slot_cap;
  const int *slot_point;
  double *state;      // state at the start of the launch
  double *state_alt;  // second buffer: a step reads one and writes the
                      // other (kernels that update in place ignore it)
  const double *wgt;
  const CompactMeta *meta;
  int *pending;         // [slot_cap]: > 0 where a lane left the fast path
  unsigned long long *counters;
  double dt;
  int nsteps;           // steps in this launch
  int steps_left;       // steps of the call left when this launch starts
  int first_launch;     // the call's first launch
};

// Sedimentation of columns (sediment.hip): point (column c, level l) is
// point c * col_stride + l * lev_stride of N [points][S*B].
constexpr int kSedMaxLevels = 64;
struct SedArgs {
  double *N;
  int64_t ncols;
  int nlev;
  int SB;
  int64_t col_stride, lev_stride;
  const double *dz;    // [nlev] layer thickness (cm)
  const double *v;     // [S*B] fall speed (cm/s)
  const double *vfac;  // [ncols][nlev] factor on the fall speed, or null
  double dt;
  int nsteps;
  double *precip;      // [ncols][S*B] number per cm^2, added to; or null
};

// Condensation/evaporation of the first species' spectrum (condense.hip).
struct CondArgs {
  double *N;               // [npoints][S*B]; bins 0..B-1 updated
  int64_t npoints;
  int SB, B, s;            // row stride, bins, bins per mass doubling
  const double *ssat;      // [npoints] supersaturation (fraction)
  const double *gcoef;     // [npoints] growth coefficient G (cm^2/s)
  double dt;
  int nsteps;
  double *evaporated;      // [npoints] g/cm^3 added to, or null
  const double *x;         // [B] bin masses (g), device
  const double *r2;        // [B] squared radii (cm^2), device
  double vol;              // x = vol r^3
  int *idx;                // [npoints] compacted points (workspace)
  int *count;              // [1] number of compacted points (workspace)
};

// --- host-side launchers (defined in the kernel translation units) -------
// nmask > 1: points are bucketed by bracket and species set (closure of
// the species holding mass), B bins per species.
hipError_t launch_compact_count(const double *N, const double *p,
                                int64_t npoints, int SB, const double *plev,
                                int L, int *block_counts,
                                unsigned char *cloudy, int nblocks,
                                const double *t_old, const double *t_now,
                                int B, int nmask,
                                const unsigned char *closure,
                                hipStream_t st);
hipError_t launch_compact_scan(const int *block_counts, int *block_offsets,
                               int nblocks, int nbuckets, CompactMeta *meta,
                               hipStream_t st);
hipError_t launch_compact_gather(const double *N, const double *p,
                                 int64_t npoints, int S, int B,
                                 const double *plev, int L,
                                 const int *block_offsets,
                                 const CompactMeta *meta, int nblocks,
                                 int *slot_point, double *state,
                                 double *wgt, int slot_cap,
                                 const double *x, double *tot, int aos,
                                 unsigned *keys, double theta,
                                 const unsigned char *cloudy, int nbuckets,
                                 hipStream_t st);
hipError_t launch_fill_padding(const CompactMeta *meta, int *slot_point,
                               unsigned *keys, int slot_cap, int nbuckets,
                               hipStream_t st);
// With keys: order the compacted slots by key within chunks, then load the
// state (tiled layout) in that order.
hipError_t launch_compact_sort_load(const double *N, const CompactMeta *meta,
                                    const unsigned *keys, int *slot_point,
                                    double *wgt, int SB, double *state,
                                    int slot_cap, hipStream_t st);
hipError_t launch_scatter(double *N, int64_t npoints, int S, int B,
                          const CompactMeta *meta, const int *slot_point,
                          const double *state, int slot_cap, const double *x,
                          double *tot, int aos, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t st);
hipError_t launch_check_state(const double *N, int64_t n, int *bad,
                              hipStream_t st);

// One-point-per-lane kernels (single species, mass-doubling grid).
bool lane_kernel_supported(int B, int S, int s);
hipError_t launch_lane_step(const StepArgs &a, int precision,
                            int waves_per_block, int max_slots,
                            hipStream_t st);
// One-point-per-wave kernels (any species set and grid), over one or more
// grids; they run the positivity limiter's second pass themselves (FP32C:
// in the FP64 follow-up launch with pending_only set).
hipError_t launch_wave_step(const WaveArgs &a, int precision, int blocks,
                            hipStream_t st);

// One-point-per-lane FP32C kernels for two to four species on the doubling
// grid (slots bucketed by bracket and species set, tiled state, double
// buffered); a point they hand over (pending) finishes the call in the
// one-point-per-wave kernel's FP64 mode.
bool multi_kernel_supported(int B, int S, int s, int nbr);
hipError_t launch_multi_step(const StepArgs &a, int max_slots,
                             hipStream_t st);

// Sedimentation steps of every (column, species-bin) pair.
hipError_t launch_sed_steps(const SedArgs &a, hipStream_t st);

// Compacts the points whose first species holds drops and whose growth is
// nonzero (a.idx, a.count), then advances them a.nsteps steps.
hipError_t launch_condense(const CondArgs &a, hipStream_t st);
bool cond_supported(int B);  // bins per species the kernel is built for

// Spontaneous breakup of the first species' spectrum (breakup.hip).
struct BrkArgs {
  double *N;         // [npoints][S*B]; bins 0..B-1 updated
  int64_t npoints;
  int SB, B;
  const double *b;   // [B] share of a bin breaking per step, device
  const double *QT;  // [B][B] fragments, transposed: QT[k][l] = Q[l][k]
  const double *Q;   // [B][B] fragments, Q[l][k] (wave kernel)
  int nsteps;
  int *idx;          // [npoints] compacted points (workspace)
  int *count;        // [1] number of compacted points (workspace)
};
hipError_t launch_breakup(const BrkArgs &a, hipStream_t st);
bool brk_supported(int B);

// Lists (idx, count) the points with a nonzero species-0 bin in kmin..B-1
// and, if ssat is given, a nonzero 2 G s dt (condense.hip).
hipError_t launch_liquid_compact(const double *N, int64_t npoints, int SB,
                                 int B, int kmin, const double *ssat,
                                 const double *gcoef, double dt, int *idx,
                                 int *count, hipStream_t st);

// One-point-per-lane kernel of the sequential (in-place) form: one species,
// mass-doubling grid, FP64; updates the state in place (a.state).
hipError_t launch_lane_seq(const StepArgs &a, int wpb, int max_slots,
                           hipStream_t st);

// Exact FP64 steps (with the positivity limiter) for every slot whose fast
// kernel stopped on an over-demand bound: once a point leaves the fast path
// it takes every remaining step of the call on the exact path, so results do
// not depend on how the call is cut into launches.  Clears pending[].
hipError_t launch_slow_steps(const StepArgs &a, int max_slots,
                             hipStream_t st);

}  // namespace fsbm
