// compact.hip -- cloudy-point compaction and the AoS <-> SoA staging around
// the step kernels.
//
// The paper isolates the collision call behind a per-point predicate array
// (Sec. VI-B) and notes that cloud-free cells need far less work (Sec. VIII).
// Here a point is cloudy iff it holds mass (and, with temperatures given,
// passes the gates of FSBM's main loop, Sec. III); collisions neither create
// nor remove a point's mass, so the cloudy set is fixed for the whole call
// and is built once per call:
//   count   per block of points: a cloudy flag per point (the block's rows
//           read with coalesced loads) and cloudy points per pressure
//           bracket
//   scan    one block: exclusive scan over blocks, per bracket; bracket
//           bases padded to whole waves so that each wave of the step
//           kernels sees a single bracket
//   gather  cloudy point (by its flag) -> slot (stable: point order within
//           a bracket),
//           bins copied into the structure-of-arrays workspace,
//           interpolation weight and FP64 totals recorded
//   sort    (one-point-per-lane kernels only) within chunks of 2048 slots,
//           points ordered by bracket, top active bin and total mass, then
//           the state is loaded in that order: a wave of the lane kernels
//           visits the union of its 64 points' active bins, and points with
//           similar top bins and similar mass (which sets how fast the top
//           bin grows) keep that union close to each point's own range
//   scatter workspace -> caller's [point][species][bin] array, totals
// Everything stays on the device, so the sequence can be captured in a
// hipGraph without host round trips.
#include <algorithm>

#include "device_common.hpp"

namespace fsbm {

namespace {

constexpr int kCompactThreads = 256;

// Temperature gates of FSBM's loop over grid points (Sec. III, main-loop
// listing): the microphysics of a point runs only where its previous
// temperature exceeds 193.15 K, and collisions within it only where the
// current temperature exceeds 223.15 K; both comparisons strict.
constexpr double kTOldMin = 193.15;
constexpr double kTCollMin = 223.15;

// Pressure bracket and weight of level l: clamp p into the tabulated range,
// take the first level pair with p_l >= p >= p_{l+1}, w is the weight of
// level l (linear interpolation, Sec. VI-A).
__device__ __forceinline__ void bracket_of(const double *plev, int L,
                                           double p, int &l, double &w) {
  if (L == 1) {
    l = 0;
    w = 0.0;
    return;
  }
  p = fmin(fmax(p, plev[L - 1]), plev[0]);
  int b = 0;
  while (b < L - 2 && !(plev[b] >= p && p >= plev[b + 1])) ++b;
  l = b;
  w = (p - plev[b + 1]) / (plev[b] - plev[b + 1]);
}

// Flag of a point in the per-point byte array left by compact_count.
constexpr unsigned char kFlagDry = 0;     // no mass
constexpr unsigned char kFlagGated = 255; // mass, stopped by a temperature
                                          // gate: unchanged, totals kept
// any other value: 1 + the point's bucket; it takes part in the call
__device__ __forceinline__ bool flag_active(unsigned char f) {
  return f != kFlagDry && f != kFlagGated;
}

// Cloudy flags and per-bucket counts of one block of points.  A point takes
// part in the call if it holds mass and passes the temperature gates
// (t_old, t_now; a null array passes its test).  Its bucket is its pressure
// bracket l, or with nmask > 1 (multi-species lane kernels) l * nmask + the
// closure of the set of species holding mass.  The block's rows are one
// contiguous run of S*B doubles per point: its threads read the run with
// consecutive addresses (one wave load covers 512 bytes) and mark the point
// of every positive entry in LDS (with nmask > 1, the entry's species bit);
// the point of entry e is e / SB, taken as the high word of e * magic with
// magic = ceil(2^32 / SB), exact for every e < 256 SB.  Then each thread
// counts its own point.
__global__ void __launch_bounds__(kCompactThreads)
    compact_count(const double *__restrict__ N, const double *__restrict__ p,
                  int64_t npoints, int SB, unsigned magic,
                  const double *__restrict__ plev, int L,
                  int *__restrict__ block_counts,
                  unsigned char *__restrict__ cloudy,
                  const double *__restrict__ t_old,
                  const double *__restrict__ t_now, int B, int nmask,
                  const unsigned char *__restrict__ closure) {
  __shared__ int cnt[kMaxBuckets];
  __shared__ unsigned char wet[kCompactThreads];
  __shared__ unsigned spec[kCompactThreads];
  const int t = threadIdx.x;
  if (t < kMaxBuckets) cnt[t] = 0;
  wet[t] = 0;
  spec[t] = 0u;
  __syncthreads();
  // the grid covers the workspace's capacity: blocks past this call's
  // points have no rows (np = 0) and count zero
  const int64_t p0 = (int64_t)blockIdx.x * kCompactThreads;
  const int np =
      (int)max((int64_t)0, min((int64_t)kCompactThreads, npoints - p0));
  const double *__restrict__ run = N + p0 * SB;
  const unsigned total = (unsigned)np * (unsigned)SB;
  // four loads in flight per thread
  for (unsigned e0 = t; e0 < total; e0 += 4 * kCompactThreads) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned e = e0 + u * kCompactThreads;
      v[u] = e < total ? run[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned e = e0 + u * kCompactThreads;
      if (v[u] > 0.0) {
        const unsigned pt = __umulhi(e, magic);
        wet[pt] = 1;
        if (nmask > 1)
          atomicOr(&spec[pt], 1u << ((e - pt * (unsigned)SB) / (unsigned)B));
      }
    }
  }
  __syncthreads();
  if (t < np) {
    const bool has_mass = wet[t] != 0;
    bool c = has_mass;
    // a NaN temperature fails its test
    if (c && t_old) c = t_old[p0 + t] > kTOldMin;
    if (c && t_now) c = t_now[p0 + t] > kTCollMin;
    unsigned char f = has_mass ? kFlagGated : kFlagDry;
    if (c) {
      int l;
      double w;
      bracket_of(plev, L, p[p0 + t], l, w);
      const int bk = nmask > 1 ? l * nmask + closure[spec[t]] : l;
      atomicAdd(&cnt[bk], 1);
      f = (unsigned char)(1 + bk);
    }
    cloudy[p0 + t] = f;
  }
  __syncthreads();
  if (t < kMaxBuckets)
    block_counts[(size_t)blockIdx.x * kMaxBuckets + t] = cnt[t];
}

// One block of 1024 threads: exclusive scan of block counts per bracket.
__global__ void __launch_bounds__(1024)
    compact_scan(const int *__restrict__ block_counts,
                 int *__restrict__ block_offsets, int nblocks, int nbuckets,
                 CompactMeta *__restrict__ meta) {
  __shared__ int part[1024];
  __shared__ int totals[kMaxBuckets];
  const int t = threadIdx.x;
  const int per = (nblocks + 1023) / 1024;
  const int b0 = t * per;
  const int b1 = min(b0 + per, nblocks);
  for (int bk = 0; bk < nbuckets; ++bk) {
    int s = 0;
    for (int b = b0; b < b1; ++b) s += block_counts[(size_t)b * kMaxBuckets + bk];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int o = 1; o < 1024; o <<= 1) {
      int v = (t >= o) ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = part[t] - s;  // exclusive prefix of this thread's range
    for (int b = b0; b < b1; ++b) {
      const int c = block_counts[(size_t)b * kMaxBuckets + bk];
      block_offsets[(size_t)b * kMaxBuckets + bk] = run;
      run += c;
    }
    if (t == 1023) totals[bk] = part[1023];
    __syncthreads();
  }
  if (t == 0) {
    int base = 0, nact = 0;
    for (int bk = 0; bk < kMaxBuckets; ++bk) {
      const int c = bk < nbuckets ? totals[bk] : 0;
      meta->bucket_base[bk] = base;
      meta->bucket_count[bk] = c;
      base += (c + kWave - 1) / kWave * kWave;
      nact += c;
    }
    meta->bucket_base[kMaxBuckets] = base;
    meta->nslots = base;
    meta->nactive = nact;
  }
}

__global__ void __launch_bounds__(kCompactThreads)
    compact_gather(const double *__restrict__ N, const double *__restrict__ p,
                   int64_t npoints, int S, int B,
                   const double *__restrict__ plev, int L,
                   const int *__restrict__ block_offsets,
                   const CompactMeta *__restrict__ meta,
                   int *__restrict__ slot_point, double *__restrict__ state,
                   double *__restrict__ wgt, int slot_cap,
                   const double *__restrict__ x, double *__restrict__ tot,
                   int aos, unsigned *__restrict__ keys, double theta,
                   const unsigned char *__restrict__ cloudy_flag,
                   int nbuckets) {
  constexpr int kWaves = kCompactThreads / kWave;
  __shared__ int wave_cnt[kWaves][kMaxBuckets];
  const int SB = S * B;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int64_t pt = (int64_t)blockIdx.x * kCompactThreads + threadIdx.x;
  const bool inside = pt < npoints;
  const double *row = N + (inside ? pt : 0) * SB;
  const unsigned char flag = inside ? cloudy_flag[pt] : kFlagDry;
  const bool cloudy = flag_active(flag);
  // gated points keep their mass: their totals are still recorded
  const bool has_mass = flag != kFlagDry;
  int l = 0, br = 0;
  double w = 0.0;
  if (cloudy) {
    bracket_of(plev, L, p[pt], br, w);
    l = flag - 1;  // the point's bucket
  }
  // stable rank of this point among the block's cloudy points of bucket l
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  int rank = 0;
  for (int bk = 0; bk < nbuckets; ++bk) {
    const uint64_t m = __ballot(cloudy && l == bk);
    if (lane == 0) wave_cnt[wv][bk] = __popcll(m);
    if (cloudy && l == bk) rank = __popcll(m & lt_mask);
  }
  __syncthreads();
  // FP64 totals of the point (one pass over its row)
  double m = 0.0, n = 0.0;
  if (has_mass)
    for (int a = 0; a < S; ++a)
      for (int k = 0; k < B; ++k) {
        const double v = row[a * B + k];
        m += v * x[k];
        n += v;
      }
  (void)br;
  if (cloudy) {
    int before = 0;
    for (int v = 0; v < wv; ++v) before += wave_cnt[v][l];
    const int slot = meta->bucket_base[l] +
                     block_offsets[(size_t)blockIdx.x * kMaxBuckets + l] +
                     before + rank;
    slot_point[slot] = (int)pt;
    wgt[slot] = w;
    if (keys) {
      // sort key: bucket, top active bin over the species, top 16 bits of
      // the total mass (positive doubles order like their bit patterns);
      // the state is loaded after the sort
      const double mt = m;
      int top = 0;
      for (int a = 0; a < S; ++a)
        for (int k = B - 1; k > top; --k)
          if (row[a * B + k] * x[k] >= theta * mt && row[a * B + k] > 0.0) {
            top = k;
            break;
          }
      const unsigned long long bits =
          (unsigned long long)__double_as_longlong(mt);
      keys[slot] = ((unsigned)l << 24) | ((unsigned)min(top, 255) << 16) |
                   (unsigned)((bits >> 48) & 0xffffu);
    } else if (aos) {
      for (int q = 0; q < SB; ++q) state[state_index_aos(q, slot, SB)] = row[q];
    } else {
      for (int q = 0; q < SB; ++q) state[state_index(q, slot, SB)] = row[q];
    }
  }
  if (inside && tot) {
    tot[pt] = m;                     // mass before
    tot[(size_t)npoints + pt] = m;   // mass after (if not stepped: unchanged)
    tot[2 * (size_t)npoints + pt] = n;
    tot[3 * (size_t)npoints + pt] = n;
  }
}

// Padding slots of each bracket (up to the next whole wave) hold no point;
// their sort key is the largest of their bracket, so a chunk sort keeps
// every bracket (with its padding) on the slots it had.
__global__ void fill_padding(const CompactMeta *__restrict__ meta,
                             int *__restrict__ slot_point,
                             unsigned *__restrict__ keys) {
  const int bk = blockIdx.x;
  const int first = meta->bucket_base[bk] + meta->bucket_count[bk];
  const int end = meta->bucket_base[bk + 1];
  const int s = first + threadIdx.x;
  if (s < end) {
    slot_point[s] = -1;
    if (keys) keys[s] = ((unsigned)bk << 24) | 0xffffffu;
  }
}

constexpr int kSortChunk = 2048;
constexpr int kSortThreads = 1024;

// Bitonic sort of one chunk of slots by key, with the point index and the
// interpolation weight carried along (deterministic: ties resolve the same
// way on every run).
__global__ void __launch_bounds__(kSortThreads)
    compact_sort(const CompactMeta *__restrict__ meta,
                 const unsigned *__restrict__ keys,
                 int *__restrict__ slot_point, double *__restrict__ wgt) {
  __shared__ unsigned ks[kSortChunk];
  __shared__ int ps[kSortChunk];
  __shared__ double ws[kSortChunk];
  const int nslots = meta->nslots;
  const int c0 = blockIdx.x * kSortChunk;
  if (c0 >= nslots) return;
  const int cnt = min(kSortChunk, nslots - c0);
  for (int t = threadIdx.x; t < kSortChunk; t += kSortThreads) {
    const bool in = t < cnt;
    ks[t] = in ? keys[c0 + t] : 0xffffffffu;
    ps[t] = in ? slot_point[c0 + t] : -1;
    ws[t] = in ? wgt[c0 + t] : 0.0;
  }
  __syncthreads();
  for (int size = 2; size <= kSortChunk; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < kSortChunk / 2; t += kSortThreads) {
        const int a = 2 * t - (t & (stride - 1));
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const unsigned ka = ks[a], kb = ks[b];
        if ((ka > kb) == up && ka != kb) {
          ks[a] = kb;
          ks[b] = ka;
          const int pa = ps[a];
          ps[a] = ps[b];
          ps[b] = pa;
          const double wa = ws[a];
          ws[a] = ws[b];
          ws[b] = wa;
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < cnt; t += kSortThreads) {
    slot_point[c0 + t] = ps[t];
    wgt[c0 + t] = ws[t];
  }
}

// Tiled staging of the one-point-per-lane paths (at most kMultiMaxSB bins
// per point): a wave moves the 64 points of one tile, each chunk of up to
// kTileBins bins of a point's row of the caller's array with one coalesced
// access (lane = bin), transposed through LDS into the tile's rows (lane =
// slot).  A bounded grid strides over the tiles, since only the device
// knows how many slots are filled.
constexpr int kTileBins = 64;
constexpr int kTilePitch = kWave + 1;  // LDS row pitch (doubles)
constexpr int kTileGridMax = 16384;

// State of every compacted point into its (sorted) slot, tiled layout;
// bins in chunks of kTileBins (lane = bin within the chunk).
__global__ void __launch_bounds__(kWave)
    compact_load(const double *__restrict__ N,
                 const CompactMeta *__restrict__ meta,
                 const int *__restrict__ slot_point, int SB,
                 double *__restrict__ state) {
  __shared__ double tile[kTileBins * kTilePitch];
  const int lane = threadIdx.x;
  const int nslots = meta->nslots;
  constexpr int kBatch = 8;  // rows whose loads are in flight together
  for (int t0 = blockIdx.x * kWave; t0 < nslots; t0 += gridDim.x * kWave) {
    for (int c0 = 0; c0 < SB; c0 += kTileBins) {
      const int q = c0 + lane;
      for (int r0 = 0; r0 < kWave; r0 += kBatch) {
        double v[kBatch];
        int pr[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int slot = t0 + r0 + u;
          pr[u] = slot < nslots ? slot_point[slot] : -1;
          v[u] = (pr[u] >= 0 && q < SB) ? N[(int64_t)pr[u] * SB + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (pr[u] >= 0 && q < SB) tile[lane * kTilePitch + r0 + u] = v[u];
      }
      __syncthreads();
      const int slot = t0 + lane;
      const int nq = min(kTileBins, SB - c0);
      if (slot < nslots && slot_point[slot] >= 0)
        for (int r = 0; r < nq; ++r)
          state[state_index(c0 + r, slot, SB)] = tile[r * kTilePitch + lane];
      __syncthreads();
    }
  }
}

// Tiled state back into the caller's array (the reverse of compact_load),
// with each point's FP64 totals after the call (species, then bins in
// ascending order).
__global__ void __launch_bounds__(kWave)
    scatter_tiled(double *__restrict__ N, int SB, int B,
                  const CompactMeta *__restrict__ meta,
                  const int *__restrict__ slot_point,
                  const double *__restrict__ state,
                  const double *__restrict__ x, double *__restrict__ tot,
                  int64_t npoints) {
  __shared__ double tile[kTileBins * kTilePitch];
  const int lane = threadIdx.x;
  const int nslots = meta->nslots;
  for (int t0 = blockIdx.x * kWave; t0 < nslots; t0 += gridDim.x * kWave) {
    const int slot = t0 + lane;
    const int pt = slot < nslots ? slot_point[slot] : -1;
    double m = 0.0, n = 0.0;
    for (int c0 = 0; c0 < SB; c0 += kTileBins) {
      const int nq = min(kTileBins, SB - c0);
      if (pt >= 0)
        for (int r = 0; r < nq; ++r) {
          const int q = c0 + r;
          const double v = state[state_index(q, slot, SB)];
          tile[r * kTilePitch + lane] = v;
          m += v * x[q % B];
          n += v;
        }
      __syncthreads();
      for (int r = 0; r < kWave; ++r) {
        const int sr = t0 + r;
        const int pr = sr < nslots ? slot_point[sr] : -1;
        if (pr >= 0 && lane < nq)
          N[(int64_t)pr * SB + c0 + lane] = tile[lane * kTilePitch + r];
      }
      __syncthreads();
    }
    if (pt >= 0 && tot) {
      tot[(size_t)npoints + pt] = m;
      tot[3 * (size_t)npoints + pt] = n;
    }
  }
}

// Workspace -> caller's array for the one-point-per-wave path (each slot's
// bins contiguous), with each point's FP64 totals after the call.
__global__ void __launch_bounds__(kCompactThreads)
    scatter_back(double *__restrict__ N, int S, int B,
                 const CompactMeta *__restrict__ meta,
                 const int *__restrict__ slot_point,
                 const double *__restrict__ state, int slot_cap,
                 const double *__restrict__ x, double *__restrict__ tot,
                 int64_t npoints, int aos) {
  const int slot = blockIdx.x * kCompactThreads + threadIdx.x;
  if (slot >= meta->nslots) return;
  const int pt = slot_point[slot];
  if (pt < 0) return;
  const int SB = S * B;
  double *row = N + (int64_t)pt * SB;
  double m = 0.0, n = 0.0;
  for (int a = 0, q = 0; a < S; ++a)
    for (int k = 0; k < B; ++k, ++q) {
      const double v = aos ? state[state_index_aos(q, slot, SB)]
                           : state[state_index(q, slot, SB)];
      row[q] = v;
      m += v * x[k];
      n += v;
    }
  if (tot) {
    tot[(size_t)npoints + pt] = m;
    tot[3 * (size_t)npoints + pt] = n;
  }
}

__global__ void zero_u64(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void check_state(const double *__restrict__ N, int64_t n,
                            int *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = N[i];
    if (!(v >= 0.0) || !isfinite(v)) atomicOr(bad, 1);
  }
}

}  // namespace

hipError_t launch_compact_count(const double *N, const double *p,
                                int64_t npoints, int SB, const double *plev,
                                int L, int *block_counts,
                                unsigned char *cloudy, int nblocks,
                                const double *t_old, const double *t_now,
                                int B, int nmask,
                                const unsigned char *closure,
                                hipStream_t st) {
  if (SB < 1 || SB > kWave * kMaxOwn ||
      npoints > (int64_t)nblocks * kCompactThreads)
    return hipErrorInvalidValue;
  const unsigned magic = 0xffffffffu / (unsigned)SB + 1u;
  hipLaunchKernelGGL(compact_count, dim3(nblocks), dim3(kCompactThreads), 0,
                     st, N, p, npoints, SB, magic, plev, L, block_counts,
                     cloudy, t_old, t_now, B, nmask, closure);
  return hipGetLastError();
}

hipError_t launch_compact_scan(const int *block_counts, int *block_offsets,
                               int nblocks, int nbuckets, CompactMeta *meta,
                               hipStream_t st) {
  hipLaunchKernelGGL(compact_scan, dim3(1), dim3(1024), 0, st, block_counts,
                     block_offsets, nblocks, nbuckets, meta);
  return hipGetLastError();
}

hipError_t launch_compact_gather(const double *N, const double *p,
                                 int64_t npoints, int S, int B,
                                 const double *plev, int L,
                                 const int *block_offsets,
                                 const CompactMeta *meta, int nblocks,
                                 int *slot_point, double *state, double *wgt,
                                 int slot_cap, const double *x, double *tot,
                                 int aos, unsigned *keys, double theta,
                                 const unsigned char *cloudy, int nbuckets,
                                 hipStream_t st) {
  hipLaunchKernelGGL(compact_gather, dim3(nblocks), dim3(kCompactThreads), 0,
                     st, N, p, npoints, S, B, plev, L, block_offsets, meta,
                     slot_point, state, wgt, slot_cap, x, tot, aos, keys,
                     theta, cloudy, nbuckets);
  return hipGetLastError();
}

hipError_t launch_fill_padding(const CompactMeta *meta, int *slot_point,
                               unsigned *keys, int slot_cap, int nbuckets,
                               hipStream_t st) {
  (void)slot_cap;
  if (nbuckets < 1 || nbuckets > kMaxBuckets) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_padding, dim3(nbuckets), dim3(kWave), 0, st,
                     meta, slot_point, keys);
  return hipGetLastError();
}

hipError_t launch_compact_sort_load(const double *N, const CompactMeta *meta,
                                    const unsigned *keys, int *slot_point,
                                    double *wgt, int SB, double *state,
                                    int slot_cap, hipStream_t st) {
  // every slot below slot_cap belongs to some chunk; chunks past the
  // compacted count return at once
  const int chunks = (slot_cap + kSortChunk - 1) / kSortChunk;
  hipLaunchKernelGGL(compact_sort, dim3(chunks), dim3(kSortThreads), 0, st,
                     meta, keys, slot_point, wgt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (SB < 1 || SB > kMultiMaxSB) return hipErrorInvalidValue;
  const int blocks = std::min((slot_cap + kWave - 1) / kWave, kTileGridMax);
  hipLaunchKernelGGL(compact_load, dim3(blocks), dim3(kWave), 0, st, N, meta,
                     slot_point, SB, state);
  return hipGetLastError();
}

hipError_t launch_scatter(double *N, int64_t npoints, int S, int B,
                          const CompactMeta *meta, const int *slot_point,
                          const double *state, int slot_cap, const double *x,
                          double *tot, int aos, hipStream_t st) {
  if (!aos) {
    // tiled layout: the one-point-per-lane paths
    if (S * B > kMultiMaxSB) return hipErrorInvalidValue;
    const int blocks =
        std::min((slot_cap + kWave - 1) / kWave, kTileGridMax);
    hipLaunchKernelGGL(scatter_tiled, dim3(blocks), dim3(kWave), 0, st, N,
                       S * B, B, meta, slot_point, state, x, tot, npoints);
    return hipGetLastError();
  }
  const int blocks = (slot_cap + kCompactThreads - 1) / kCompactThreads;
  hipLaunchKernelGGL(scatter_back, dim3(blocks), dim3(kCompactThreads), 0, st,
                     N, S, B, meta, slot_point, state, slot_cap, x, tot,
                     npoints, aos);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_check_state(const double *N, int64_t n, int *bad,
                              hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(check_state, dim3((unsigned)blocks), dim3(256), 0, st, N,
                     n, bad);
  return hipGetLastError();
}

}  // namespace fsbm
