// kernels_seq.hip -- one grid point per lane: the collision step in the
// sequential form of Bott's flux method (one species, mass-doubling grid).
//
// The sequential form takes the bin pairs one after another, i ascending
// and then j = i..B-1, and moves mass in place: each pair sees what the
// pairs before it left.  Positivity needs no second pass: the collisions
// of a pair are capped so that bin i gives at most what it holds (half of
// it for the pair (i, i)), and the flux out of the target at what the
// target then holds.  A capped bin is left exactly empty (its exact-
// arithmetic value), so that no rounding residue takes part in later
// pairs, where a pair (i, j) would scale it by 2^(j-i).  On the doubling
// grid (x_{k+1} = 2 x_k) the merged mass of a pair i < j lands in bin j
// itself, so bin j is never a losing source and takes no cap; the pair
// (i, i) lands exactly on bin i+1 with no flux.
//
// Mapping (gfx950):
//  * the masses of the lane's point stay in VGPRs for all steps of the
//    launch (static register indices: bins j are unrolled); the state is
//    read from the tiled workspace once at the start of the launch and
//    written back at its end;
//  * rows i are wave-uniform and run in order, skipped when no lane of the
//    wave holds an active bin i; within a row the pairs (i, j) are skipped
//    when no lane has both bins active;
//  * the row bin's mass lives in one register during its row (read at the
//    row start and written at its end by the uniform row index); the self
//    pair's merged mass is added to bin i+1 right before the pair (i, i+1);
//  * kernel-table rows [i][j] and Courant numbers are scalar loads; every
//    wave lies in one pressure bracket.
// FP64 throughout.  Between steps the state passes through numbers
// (N = M / x, negative round-off set to zero) as the step is defined.
#include <float.h>

#include "device_common.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

template <int B, int WPB>
__global__ void __launch_bounds__(kWave *WPB)
    __attribute__((amdgpu_waves_per_eu(2))) lane_seq_f64(StepArgs a) {
  constexpr int nthr = kWave * WPB;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int slot = blockIdx.x * nthr + tid;
  const int nslots = uniform(a.meta->nslots);
  const int wave_first = uniform(slot & ~(kWave - 1));
  if (wave_first >= nslots) return;
  int br = 0;
  for (int b = 1; b < a.m.nbr; ++b)
    if (wave_first >= a.meta->bucket_base[b]) br = b;
  br = uniform(br);
  const bool live = slot < nslots && a.slot_point[slot] >= 0;
  const double w = live ? a.wgt[slot] : 0.0;
  // kernel tables [i][j][2] = (K_{l+1}, K_l - K_{l+1}) of the wave's
  // bracket; Courant numbers [i][j]
  const double *__restrict__ Kd = a.m.Kd + (size_t)br * B * B * 2;
  const double *__restrict__ ctab = a.m.ct;
  const double *__restrict__ ixg = a.m.invx;
  // doubling grid: x_k = x_1 2^k exactly
  const double x1 = ldc(a.m.x);
  double *const stw = a.state + (size_t)wave_first * B;
  const double theta = a.m.theta, dt = a.dt;
  unsigned long long npairs = 0, ncapped = 0;

  BinsD<B> M;
#pragma unroll
  for (int k = 0; k < B; ++k) {
    const double v = live ? stw[k * kWave + lane] : 0.0;
    M.set(k, ldexp(v * x1, k));
  }

  for (int step = 0; step < a.nsteps; ++step) {
    double Mtot = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) Mtot = Mtot + M.get(k);
    const double thr = theta * Mtot;

    // the pair (B-1, B-1) leaves the grid: row B-1 has no pair
    for (int i = 0; i < B - 1; ++i) {
      double mi = 0.0;
#pragma unroll
      for (int q = 0; q < B - 1; ++q)
        if (q == i) mi = M.get(q);
      if (!__any(mi > 0.0 && mi >= thr)) continue;
      const double *Ki = Kd + (size_t)i * B * 2;
      const double *ci = ctab + (size_t)i * B;
      const double ixi = ldc(ixg + i);
      // self pair: C = dt K N_i^2 / 2, at most N_i / 2; 2 C x_i moves to
      // bin i+1 (an exact hit: no flux); a kernel entry that is zero at
      // every level collides nothing
      double gain = 0.0;
      const uint64_t nzi = ldc(a.m.nzT + i);
      if ((nzi >> i) & 1ull) {
        const bool act = mi > 0.0 && mi >= thr;
        const double K = fma(ldc(Ki + i * 2 + 1), w, ldc(Ki + i * 2));
        const double Ni = mi * ixi;
        double C = ((dt * K) * Ni) * Ni;
        C = 0.5 * C;
        const double cap = 0.5 * Ni;
        const bool hit = C > cap;
        C = hit ? cap : C;
        if (act) {
          const double A = ldexp(C * x1, i);
          const double Sm = A + A;
          // a capped bin gives all it holds: exactly nothing is left
          mi = hit ? 0.0 : mi - Sm;
          gain = Sm;
          ++npairs;
          ncapped += hit ? 1u : 0u;
        }
      }
#pragma unroll
      for (int j = 1; j < B; ++j) {
        if (j <= i) continue;  // uniform
        double Mj = M.get(j);
        if (j == i + 1) Mj = Mj + gain;
        const bool act =
            mi > 0.0 && mi >= thr && Mj > 0.0 && Mj >= thr;
        if (__any(act)) {
          const double K = fma(ldc(Ki + j * 2 + 1), w, ldc(Ki + j * 2));
          const double Ni = mi * ixi;
          const double Nj = Mj * ldc(ixg + j);
          double C = ((dt * K) * Ni) * Nj;
          const bool hit = C > Ni;  // bin j receives the merged mass
          C = hit ? Ni : C;
          // A = C x_i leaves bin i; the merged mass A + Bm enters bin j,
          // which gave Bm = A 2^(j-i): bin j's content becomes M_j + A
          const double A = ldexp(C * x1, i);
          const double Sm = A + ldexp(A, j - i);
          const double Mk = Mj + A;
          double F = 0.0;
          bool fhit = false;
          if (j <= B - 2) {
            const double Mn = M.get(j + 1);
            const double x1f = fmax(log_f64(Mn / Mk), kX1Floor);
            F = flux_fraction_f64(ldc(ci + j), x1f) * Sm;
            fhit = F > Mk;
            F = fhit ? Mk : F;
            if (act) M.set(j + 1, Mn + F);
          }
          if (act) {
            mi = hit ? 0.0 : mi - A;
            Mj = Mk - F;
            ++npairs;
            ncapped += (hit || fhit) ? 1u : 0u;
          }
        }
        M.set(j, Mj);
      }
#pragma unroll
      for (int q = 0; q < B - 1; ++q)
        if (q == i) M.set(q, mi);
    }

    // back to numbers and masses, as the step is defined on numbers
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const double Mk = M.get(k);
      const double Nk = ldexp((Mk < 0.0 ? 0.0 : Mk) / x1, -k);
      M.set(k, ldexp(Nk * x1, k));
    }
  }

  if (live) {
#pragma unroll
    for (int k = 0; k < B; ++k)
      stw[k * kWave + lane] = ldexp(M.get(k) / x1, -k);
  }
  npairs = wave_sum_u64(npairs);
  ncapped = wave_sum_u64(ncapped);
  if (lane == 0) {
    if (npairs) atomicAdd(&a.counters[0], npairs);
    if (ncapped) atomicAdd(&a.counters[1], ncapped);
  }
}

template <int B, int WPB>
hipError_t launch_bw(const StepArgs &a, int max_slots, hipStream_t st) {
  constexpr int threads = kWave * WPB;
  const int blocks = (max_slots + threads - 1) / threads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((lane_seq_f64<B, WPB>), dim3(blocks), dim3(threads), 0,
                     st, a);
  return hipGetLastError();
}

template <int B>
hipError_t launch_b(const StepArgs &a, int wpb, int max_slots,
                    hipStream_t st) {
  if (wpb == 2) return launch_bw<B, 2>(a, max_slots, st);
  return launch_bw<B, 1>(a, max_slots, st);
}

}  // namespace

hipError_t launch_lane_seq(const StepArgs &a, int wpb, int max_slots,
                           hipStream_t st) {
  switch (a.m.B) {
    case 3:
      return launch_b<3>(a, wpb, max_slots, st);
    case 8:
      return launch_b<8>(a, wpb, max_slots, st);
    case 16:
      return launch_b<16>(a, wpb, max_slots, st);
    case 33:
      return launch_b<33>(a, wpb, max_slots, st);
    case 40:
      return launch_b<40>(a, wpb, max_slots, st);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fsbm
