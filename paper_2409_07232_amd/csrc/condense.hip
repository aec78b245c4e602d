// condense.hip -- condensation and evaporation of the drop spectrum (the
// first species) at a prescribed supersaturation per point.  Over a step
// every drop of bin k grows by r dr/dt = G s, so its r^2 grows by 2 G s dt
// exactly; its number is then shared between the two grid bins around the
// new mass so that number and mass are both kept.  Drops whose r^2 falls to
// zero, or whose new mass lies below the grid, evaporate (their mass is
// reported per point); drops that grow past the grid stay in the last bin.
// The paper lists this process in the bin equation (Sec. III, eq. (1)) and
// names it as the next part to offload (Sec. VIII); the growth law and the
// number-and-mass remapping are the published ones (Rogers and Yau 1989,
// ch. 7; Kovetz and Olund 1969).
//
// Mapping (gfx950):
//  * compaction: one pass over the points, each block reading its points'
//    bins as contiguous runs, flags those with drops and a nonzero growth
//    and appends them to an index list (one atomic per wave); the list's
//    order does not matter, every point is independent;
//  * one compacted point per lane; its B bins in VGPRs for all steps of the
//    call (static indices after unrolling), the receiving spectrum of a
//    step in the lane's own column of LDS (a drop's target bin is per-lane
//    data); the lane's columns are 64 doubles apart, so every access of a
//    wave hits 64 distinct banks whatever the bins;
//  * a bin's target and weight depend only on the bin and the point's
//    growth, so at 33 bins they are found once per call and held in VGPRs
//    (a step is then two multiply-adds into LDS per bin); at 66 bins they
//    are found again at every step;
//  * the target bin j (x_j <= x' < x_{j+1}) from the binary exponents of x'
//    and x_0, then corrected against the grid held in LDS: the unique bin,
//    found in at most 2 s comparisons;
//  * FP64 throughout, the definition's operations in its order, the square
//    root and the division rounded to nearest as IEEE 754 defines them, so
//    the result is the definition's bit for bit.
#include "device_common.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

constexpr int kCondThreads = 64;

__global__ void __launch_bounds__(64) cond_clear(int *count) { *count = 0; }

// Square root rounded to nearest.  The device library's FP64 square root
// is faithful (within one unit in the last place) but not always the
// nearest double; with the exact residual r = x - y^2 (one fma) Tuckerman's
// test moves y to the neighbour whose rounding interval holds sqrt(x):
// up if x > (y + u/2)^2, i.e. r > y u, down if x < (y - d/2)^2, i.e.
// r <= -y d (u, d the spacing above and below y; r, y u and y d are
// multiples of d^2, so the quarter-spacing terms drop out).
__device__ __forceinline__ double sqrt_rn(double x) {
  const double y = sqrt(x);
  const int e = ilogb(y);
  const double u = ldexp(1.0, e - 52);
  const double d = (y == ldexp(1.0, e)) ? 0.5 * u : u;
  const double r = fma(-y, y, x);
  if (r > y * u) return y + u;
  if (r <= -(y * d)) return y - d;
  return y;
}

struct CompactArgs {
  const double *N;
  int64_t npoints;
  int SB, B, kmin;
  uint32_t magic;              // ceil(2^32 / (B - kmin))
  const double *ssat, *gcoef;  // null: no growth test
  double dt;
  int *idx, *count;
};

constexpr int kCompactThreads = 256;
constexpr int kCompactPoints = 1024;  // points per block (4 per thread)
constexpr int kCompactWaves = kCompactThreads / kWave;
constexpr int kCompactRounds = kCompactPoints / kCompactThreads;

// Appends the points with drops in bins kmin..B-1 (and a nonzero growth
// where one is given).  A block takes 1024 consecutive points and reads
// their bins kmin..B-1 as runs of consecutive addresses across its lanes
// (element e is point e / (B - kmin), found with a multiply-high; exact for
// e < 2^32 / B), marking the points with drops in LDS; the block then
// claims room for all its listed points with one atomic.
__global__ void __launch_bounds__(kCompactThreads) liquid_compact(
    CompactArgs a) {
  __shared__ unsigned char held[kCompactPoints];
  __shared__ int part[kCompactRounds * kCompactWaves];
  __shared__ int bbase;
  const int tid = threadIdx.x;
  const int64_t first = (int64_t)blockIdx.x * kCompactPoints;
  for (int i = tid; i < kCompactPoints; i += kCompactThreads) held[i] = 0;
  __syncthreads();
  const int nb = a.B - a.kmin;
  const int npt = (int)min<int64_t>(kCompactPoints, a.npoints - first);
  const double *base = a.N + first * a.SB + a.kmin;
  // eight loads in flight per thread before their tests; elements past
  // the block's last one read that one again (in bounds) and are ignored
  const int ne = npt * nb;
  for (int e0 = tid; e0 < ne; e0 += 8 * kCompactThreads) {
    double v[8];
    int pp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * kCompactThreads, ne - 1);
      pp[u] = (int)__umulhi((unsigned)e, a.magic);
      v[u] = base[(int64_t)pp[u] * a.SB + (e - pp[u] * nb)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] != 0.0) held[pp[u]] = 1;
  }
  __syncthreads();
  const int lane = tid & (kWave - 1), w = tid / kWave;
  bool act[kCompactRounds];
  uint64_t bal[kCompactRounds];
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r) {
    const int p = r * kCompactThreads + tid;
    const int64_t pt = first + p;
    act[r] = p < npt && held[p] &&
             (a.ssat ? (2.0 * a.gcoef[pt] * a.ssat[pt] * a.dt) != 0.0 : true);
    bal[r] = __ballot(act[r]);
    if (lane == 0) part[r * kCompactWaves + w] = __popcll(bal[r]);
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < kCompactRounds * kCompactWaves; ++i) {
      const int c = part[i];
      part[i] = run;
      run += c;
    }
    bbase = run ? atomicAdd(a.count, run) : 0;
  }
  __syncthreads();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r)
    if (act[r])
      a.idx[bbase + part[r * kCompactWaves + w] +
            __popcll(bal[r] & below)] =
          (int)(first + r * kCompactThreads + tid);
}

template <int B>
__global__ void __launch_bounds__(kCondThreads) cond_steps(CondArgs a) {
  __shared__ double nn[B * kCondThreads];
  __shared__ double xs[B];
  const int count = *a.count;
  if ((int64_t)blockIdx.x * kCondThreads >= count) return;  // whole block
  const int tid = threadIdx.x;
  for (int k = tid; k < B; k += kCondThreads) xs[k] = a.x[k];
  __syncthreads();
  const int slot = blockIdx.x * kCondThreads + tid;
  if (slot >= count) return;
  const int64_t pt = a.idx[slot];
  double *row = a.N + pt * a.SB;
  const double growth = 2.0 * a.gcoef[pt] * a.ssat[pt] * a.dt;
  double n[B];
#pragma unroll
  for (int k = 0; k < B; ++k) n[k] = row[k];
  double *col = nn + tid;  // bin k of this lane at col[k * 64]
  const double vol = a.vol;
  const double x0 = ldc(a.x), xtop = ldc(a.x + B - 1);
  const int e0 = ilogb(x0);
  const int s = a.s;
  double evap = a.evaporated ? a.evaporated[pt] : 0.0;
  // a bin's new mass, and so its target and weight, depend only on the bin
  // and the point's growth, the same at every step of the call: found once
  // (target -1: the drops evaporate; B - 1: past the grid's top)
  auto target = [&](int k, double &phi) -> int {
    const double rr = ldc(a.r2 + k) + growth;
    if (!(rr > 0.0)) return -1;  // r^2 reaches zero
    const double xn = vol * (rr * sqrt_rn(rr));
    if (xn < x0) return -1;  // below the grid
    if (xn >= xtop) return B - 1;
    // x_{s (e - e0 - 1)} <= xn: a lower bound within 2 s bins of j
    int j = s * (ilogb(xn) - e0 - 1);
    j = j < 0 ? 0 : (j > B - 2 ? B - 2 : j);
    while (j > 0 && xs[j] > xn) --j;
    while (j < B - 2 && !(xs[j + 1] > xn)) ++j;
    const double xj = xs[j], xj1 = xs[j + 1];
    phi = (xn - xj) / (xj1 - xj);
    return j;
  };
  constexpr bool kHold = B <= 40;  // targets and weights held in VGPRs
  int tj[kHold ? B : 1];
  double ph[kHold ? B : 1];
  if (kHold) {
#pragma unroll
    for (int k = 0; k < B; ++k) {
      ph[kHold ? k : 0] = 0.0;
      tj[kHold ? k : 0] = target(k, ph[kHold ? k : 0]);
    }
  }
  for (int st = 0; st < a.nsteps; ++st) {
#pragma unroll
    for (int k = 0; k < B; ++k) col[k * kCondThreads] = 0.0;
    double ev = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const double nk = n[k];
      if (nk == 0.0) continue;
      double phi = 0.0;
      const int j = kHold ? tj[kHold ? k : 0] : target(k, phi);
      if (kHold) phi = ph[kHold ? k : 0];
      if (j < 0) {
        ev += nk * ldc(a.x + k);
      } else if (j == B - 1) {
        col[(B - 1) * kCondThreads] += nk;
      } else {
        col[j * kCondThreads] += nk * (1.0 - phi);
        col[(j + 1) * kCondThreads] += nk * phi;
      }
    }
#pragma unroll
    for (int k = 0; k < B; ++k) n[k] = col[k * kCondThreads];
    evap += ev;
  }
#pragma unroll
  for (int k = 0; k < B; ++k) row[k] = n[k];
  if (a.evaporated) a.evaporated[pt] = evap;
}

// Grids beyond the lane kernels (67 to kMaxBins bins): one listed point
// per wave at a time (a grid of waves strides over the list), its bins in
// LDS.  The bins' targets and weights are found once per call, one bin per
// lane; targets rise with the source bin (-1 for evaporating sources, a
// prefix; B - 1 for sources past the top, a suffix), so the sources that
// bin m receives from -- targets max(m - 1, 0) and m -- are one contiguous
// run, found by bisection.  Each step, lane r forms bins r, r + 64, ... by
// adding its run's contributions in ascending source order, as the
// definition adds them; the first lane sums the evaporated mass of the
// evaporating prefix in order.
__global__ void __launch_bounds__(kCondThreads) cond_wave(CondArgs a) {
  extern __shared__ double lds[];
  const int B = a.B, lane = threadIdx.x;
  double *n = lds, *nn = lds + B, *ph = lds + 2 * B, *xs = lds + 3 * B;
  int *tj = (int *)(lds + 4 * B);
  int *r0 = tj + B, *r1 = r0 + B;
  for (int k = lane; k < B; k += kCondThreads) xs[k] = a.x[k];
  __syncthreads();
  const double vol = a.vol, x0 = xs[0], xtop = xs[B - 1];
  const int e0 = ilogb(x0), s = a.s;
  const int count = *a.count;
  for (int slot = blockIdx.x; slot < count; slot += gridDim.x) {
    const int64_t pt = a.idx[slot];
    double *row = a.N + pt * a.SB;
    const double growth = 2.0 * a.gcoef[pt] * a.ssat[pt] * a.dt;
    for (int k = lane; k < B; k += kCondThreads) {
      n[k] = row[k];
      double phi = 0.0;
      int t;
      const double rr = a.r2[k] + growth;
      if (!(rr > 0.0)) {
        t = -1;  // r^2 reaches zero
      } else {
        const double xn = vol * (rr * sqrt_rn(rr));
        if (xn < x0) {
          t = -1;  // below the grid
        } else if (xn >= xtop) {
          t = B - 1;  // past the grid's top
        } else {
          int j = s * (ilogb(xn) - e0 - 1);
          j = j < 0 ? 0 : (j > B - 2 ? B - 2 : j);
          while (j > 0 && xs[j] > xn) --j;
          while (j < B - 2 && !(xs[j + 1] > xn)) ++j;
          phi = (xn - xs[j]) / (xs[j + 1] - xs[j]);
          t = j;
        }
      }
      tj[k] = t;
      ph[k] = phi;
    }
    __syncthreads();
    for (int m = lane; m < B; m += kCondThreads) {
      // first source with target >= max(m - 1, 0), first with target > m
      const int lo_t = m > 0 ? m - 1 : 0;
      int a0 = 0, b0 = B;
      while (a0 < b0) {
        const int c = (a0 + b0) >> 1;
        if (tj[c] >= lo_t) b0 = c; else a0 = c + 1;
      }
      int a1 = a0, b1 = B;
      while (a1 < b1) {
        const int c = (a1 + b1) >> 1;
        if (tj[c] > m) b1 = c; else a1 = c + 1;
      }
      r0[m] = a0;
      r1[m] = a1;
    }
    int nev = 0;  // evaporating sources: the prefix with target -1
    while (nev < B && tj[nev] < 0) ++nev;
    double evap = a.evaporated ? a.evaporated[pt] : 0.0;
    __syncthreads();
    for (int st = 0; st < a.nsteps; ++st) {
      for (int m = lane; m < B; m += kCondThreads) {
        double acc = 0.0;
        for (int k = r0[m]; k < r1[m]; ++k) {
          const double nk = n[k];
          if (nk == 0.0) continue;
          const int t = tj[k];
          if (t == m)
            acc += (m == B - 1) ? nk : nk * (1.0 - ph[k]);
          else
            acc += nk * ph[k];
        }
        nn[m] = acc;
      }
      if (lane == 0) {
        double ev = 0.0;
        for (int k = 0; k < nev; ++k)
          if (n[k] != 0.0) ev += n[k] * xs[k];
        evap += ev;
      }
      __syncthreads();
      for (int k = lane; k < B; k += kCondThreads) n[k] = nn[k];
      __syncthreads();
    }
    for (int k = lane; k < B; k += kCondThreads) row[k] = n[k];
    if (lane == 0 && a.evaporated) a.evaporated[pt] = evap;
    __syncthreads();
  }
}

template <int B>
hipError_t launch_b(const CondArgs &a, unsigned blocks, hipStream_t st) {
  hipLaunchKernelGGL(cond_steps<B>, dim3(blocks), dim3(kCondThreads), 0, st,
                     a);
  return hipGetLastError();
}

}  // namespace

bool cond_supported(int B) {
  return B == 33 || B == 66 || (B > 66 && B <= kMaxBins);
}

hipError_t launch_liquid_compact(const double *N, int64_t npoints, int SB,
                                 int B, int kmin, const double *ssat,
                                 const double *gcoef, double dt, int *idx,
                                 int *count, hipStream_t st) {
  if (npoints > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cond_clear, dim3(1), dim3(64), 0, st, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || npoints == 0) return e;
  if (kmin < 0 || kmin >= B) return hipErrorInvalidValue;
  const uint32_t nb = (uint32_t)(B - kmin);
  const uint32_t magic = (uint32_t)((0x100000000ull + nb - 1) / nb);
  CompactArgs c{N, npoints, SB, B, kmin, magic, ssat, gcoef, dt, idx, count};
  const unsigned blocks =
      (unsigned)((npoints + kCompactPoints - 1) / kCompactPoints);
  hipLaunchKernelGGL(liquid_compact, dim3(blocks), dim3(kCompactThreads), 0,
                     st, c);
  return hipGetLastError();
}

hipError_t launch_condense(const CondArgs &a, hipStream_t st) {
  if (!cond_supported(a.B) || a.s < 1 || a.npoints > 0x7fffffffLL)
    return hipErrorInvalidValue;
  if (a.npoints == 0 || a.nsteps == 0) return hipSuccess;
  hipError_t e = launch_liquid_compact(a.N, a.npoints, a.SB, a.B, 0, a.ssat,
                                       a.gcoef, a.dt, a.idx, a.count, st);
  if (e != hipSuccess) return e;
  const unsigned blocks =
      (unsigned)((a.npoints + kCondThreads - 1) / kCondThreads);
  if (a.B > 66) {
    const unsigned waves = (unsigned)(a.npoints < 2048 ? a.npoints : 2048);
    const size_t lds = (sizeof(double) * 4 + sizeof(int) * 3) * (size_t)a.B;
    hipLaunchKernelGGL(cond_wave, dim3(waves), dim3(kCondThreads), lds, st,
                       a);
    return hipGetLastError();
  }
  return a.B == 33 ? launch_b<33>(a, blocks, st) : launch_b<66>(a, blocks, st);
}

}  // namespace fsbm
