// kernels_lane.hip -- one grid point per lane: the collision step for one
// species on the mass-doubling grid (x_{k+1} = 2 x_k) with at most
// kLaneMaxBins bins.  This is the shape of the FSBM liquid spectrum with 33
// bins (Sec. III).
//
// Layout and mapping (gfx950):
//  * compacted cloudy points sit in a structure-of-arrays workspace
//    state[bin][slot], so a wave reads and writes each bin of its 64 points
//    as one contiguous 512-byte row; there are two such buffers and each
//    step reads one and writes the other;
//  * the pair loop is wave-uniform: rows j (the larger bin) run over the
//    union of the wave's active bins, in descending order; columns i < j are
//    unrolled.  Kernel-table entries, Courant numbers and bin masses are
//    therefore scalar operands, and every per-pair register access has a
//    static index (the column bin i);
//  * per lane, the masses and the losses of column bins stay in VGPRs;
//  * descending rows complete each bin's losses before its own row ends, so
//    the positivity-limiter test of a bin is taken right there, and bin j+1
//    is final after row j: its update is written out during the sweep and
//    only one gain is carried from row to row (no LDS);
//  * every wave lies in one pressure bracket (the compaction pads brackets to
//    whole waves): the per-pair kernel interpolation is one FMA with two
//    scalar table operands.
//
// Pair (i < j) on the doubling grid: target bin k = j, Courant number
// c = 2^(i-j); self pairs (j, j) land exactly on bin j+1.
//  * FP64 kernel: the method as defined, in FP64.
//  * FP32C kernel: masses normalised by the point's FP64 total; pair amounts
//    in FP32, applied as exact transfers (bin i -> bin j: A, bin j -> bin
//    j+1: F and the self-pair mass) into per-bin sums held in FP64, then
//    carried into an FP64 update of the FP64 state.  Each FP32 amount
//    enters its sums exactly; an FP64 add issues at the rate of an FP32 one
//    on CDNA, so the widened sum (convert + add) costs a third of an FP32
//    compensated one (max, min, add, sub, sub, add) and is more accurate.
// A lane whose over-demand test fires leaves the fast kernel; the exact FP64
// path (slow_path.hpp) takes the rest of the call's steps for it.
#include <float.h>

#include "device_common.hpp"
#include "slow_path.hpp"

// The exact-transfer bookkeeping relies on every rounding being the one
// written; fused forms are spelled out where wanted.
#pragma clang fp contract(off)

namespace fsbm {

namespace {

// Bracket of a wave: the compaction pads every bracket to whole waves.
__device__ __forceinline__ int wave_bracket(const CompactMeta *meta,
                                           int wave_first_slot, int nbr) {
  int br = 0;
  for (int b = 1; b < nbr; ++b)
    if (wave_first_slot >= meta->bucket_base[b]) br = b;
  return uniform(br);
}

__device__ __forceinline__ void add_counters(unsigned long long *counters,
                                             unsigned long long pairs) {
  pairs = wave_sum_u64(pairs);
  if ((threadIdx.x & (kWave - 1)) == 0 && pairs)
    atomicAdd(&counters[0], pairs);
}

// Pairs a lane evaluates in row j: bin j active, each active i < j, plus the
// self pair while its merged mass stays on the grid, all with a kernel entry
// that is nonzero at some level (row mask nz).
template <int B>
__device__ __forceinline__ unsigned row_pairs(uint64_t act, uint64_t nz,
                                              int j) {
  if (!((act >> j) & 1ull)) return 0u;
  const uint64_t below = (j == 0) ? 0ull : (act & nz & (~0ull >> (64 - j)));
  return (unsigned)__popcll(below) +
         ((j + 1 <= B - 1 && ((nz >> j) & 1ull)) ? 1u : 0u);
}

__device__ __forceinline__ bool bit_of(uint32_t lo, uint32_t hi, int k) {
  return (k < 32) ? ((lo >> k) & 1u) : ((hi >> (k - 32)) & 1u);
}

// ---------------------------------------------------------- FP64 kernel
// Both lane kernels read the step's state from one buffer and write the
// updated bins to the other.  Bin k's net change is complete once the rows
// above it and the row below it are done: its gains come from row k (mass
// arriving from smaller partners) and row k-1 (flux and self-pair mass), its
// losses as the smaller partner from the rows above.  The descending sweep
// therefore finishes bin j+1 right after row j, carrying only bin j+1's
// own-row gain from one row to the next; nothing is staged in LDS.  A lane
// that stops for the exact path copies its untouched state over, so it is
// valid in both buffers.
template <int B, int WPB>
__global__ void __launch_bounds__(kWave *WPB)
    __attribute__((amdgpu_waves_per_eu(B <= 33 ? 2 : 1))) lane_step_f64(
        StepArgs a) {
  constexpr int nthr = kWave * WPB;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int slot = blockIdx.x * nthr + tid;
  const int nslots = uniform(a.meta->nslots);
  const int wave_first = uniform(slot & ~(kWave - 1));
  if (wave_first >= nslots) return;
  const int br = wave_bracket(a.meta, wave_first, a.m.nbr);
  // a slot handed to the exact path earlier in the call stays there
  bool live = slot < nslots && a.slot_point[slot] >= 0 && a.pending[slot] == 0;
  const double w = live ? a.wgt[slot] : 0.0;
  // tables transposed to [j][i]: the columns of row j are contiguous
  const double *__restrict__ Kd = a.m.KdT + (size_t)br * B * B * 2;
  const double *__restrict__ ctab = a.m.ctT;
  const double *__restrict__ ixg = a.m.invx;
  // doubling grid: x_k = x_1 2^k exactly, so products with x_k are exact
  // power-of-two scalings of products with x_1
  const double x1 = ldc(a.m.x);
  // bin k of this lane's point: stw[k * 64 + lane] (wave tile, uniform base)
  double *const stw0 = a.state + (size_t)wave_first * B;
  double *const stw1 = a.state_alt + (size_t)wave_first * B;
  const double theta = a.m.theta, dt = a.dt;
  unsigned long long npairs = 0;

  for (int step = 0; step < a.nsteps; ++step) {
    // Opaque per-step copies of the wave's base pointers: keep the compiler
    // from hoisting B per-lane 64-bit addresses out of the step loop (the
    // accesses use a scalar base, one lane offset and immediate offsets).
    double *sb = (step & 1) ? stw1 : stw0;  // read
    double *so = (step & 1) ? stw0 : stw1;  // written
    asm volatile("" : "+s"(sb));
    asm volatile("" : "+s"(so));
    // S1/S2: masses, FP64 total (bins ascending), activity.
    BinsD<B> Mt;
    double Mtot = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const double v = sb[k * kWave + lane];
      const double Mk = live ? ldexp(__dmul_rn(v, x1), k) : 0.0;
      Mt.set(k, Mk);
      Mtot = __dadd_rn(Mtot, Mk);
    }
    const double thr = theta * Mtot;
    uint64_t act = 0;
    BinsD<B> L;  // losses of bins as the smaller partner of a pair
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const double Mk = Mt.get(k);
      const bool ak = Mk > 0.0 && Mk >= thr;
      act |= (uint64_t)ak << k;
      Mt.set(k, ak ? Mk : 0.0);
      L.set(k, 0.0);
    }
    const uint64_t uni = wave_or64(act);
    const int lo = uniform(uni ? (int)__builtin_ctzll(uni) : 0);
    const int hi = uniform(uni ? 63 - (int)__builtin_clzll(uni) : -1);
    const uint32_t uni_lo = uniform((int)(uint32_t)uni);
    const uint32_t uni_hi = uniform((int)(uint32_t)(uni >> 32));
    bool flag = false;
    unsigned step_pairs = 0;
    // S6 for bin k: FP64 update, negative round-off clamped, back to
    // numbers, into the other buffer
    auto finish = [&](int k, double g, double Nk) {
      const double Mk = ldexp(__dmul_rn(Nk, x1), k);
      double Mn = Mk + (g - L.get(k));
      Mn = Mn < 0.0 ? 0.0 : Mn;
      if (live) so[k * kWave + lane] = ldexp(Mn / x1, -k);
    };
    double g = 0.0;  // gain of bin j+1 from its own row, carried down
    // state of bin j+1, loaded one row ahead of its update (rows run over
    // the union [lo, hi] of the wave's active bins; bins lo..hi+1 change)
    double Nnext = (hi + 1 <= B - 1) ? sb[(hi + 1) * kWave + lane] : 0.0;

    // S3/S4: rows j descending, columns i < j unrolled.
    for (int j = hi; j >= lo; --j) {
      const double Nj1 = Nnext;
      Nnext = sb[j * kWave + lane];
      double gj = 0.0;  // gain of bin j from row j
      if (bit_of(uni_lo, uni_hi, j)) {
        // columns to visit: i < j with bin i active in some lane and a
        // kernel entry that is not zero at every level
        const uint64_t nz = ldc(a.m.nzT + j);
        const uint64_t below_mask =
            ((j == 0) ? 0ull : (~0ull >> (64 - j))) & nz;
        const uint32_t cl = uni_lo & (uint32_t)below_mask;
        const uint32_t ch = uni_hi & (uint32_t)(below_mask >> 32);
        const double Mtj = Mt.get(j);
        const double qj = dt * (Mtj * ldc(ixg + j));  // dt N_j, 0 if inactive
        const bool has_flux = j <= B - 2;
        const double lnj1 = has_flux ? log_f64(Mt.get(j + 1)) : 0.0;  // -inf if 0
        const double *Kj = Kd + (size_t)j * B * 2;  // row j: [i][2]
        const double *cj = ctab + (size_t)j * B;
        double netj = 0.0, fout = 0.0, dneg = 0.0;
#pragma unroll
        for (int i = 0; i < B - 1; ++i) {
          if (!bit_of(cl, ch, i)) continue;
          const double *e = Kj + i * 2;
          const double K = fma(ldc(e + 1), w, ldc(e));
          // A = C x_i = dt K N_j M_i, B = C x_j = A 2^(j-i)
          const double A = (qj * K) * Mt.get(i);
          const double Bm = ldexp(A, j - i);
          const double Sm = A + Bm;
          double F = 0.0;
          if (has_flux) {
            const double den = fmax(Mtj + Sm, DBL_MIN);
            const double x1f = fmax(lnj1 - log_f64(den), kX1Floor);
            F = flux_fraction_f64(ldc(cj + i), x1f) * Sm;
          }
          L.set(i, L.get(i) + A);
          // merged net of bin j: keeps Sm - F, loses Bm
          const double cn = A - F;
          netj += cn;
          fout += F;
          dneg += fmax(-cn, 0.0);
        }
        // self pair: 2 x_j = x_{j+1} exactly, no flux; off grid for j = B-1
        double self2 = 0.0;
        if (j + 1 <= B - 1 && ((nz >> j) & 1ull)) {
          const double *e = Kj + j * 2;
          const double K = fma(ldc(e + 1), w, ldc(e));
          const double A = 0.5 * ((qj * K) * Mtj);
          self2 = A + A;
        }
        // S5 test: demand on bin j = its losses as the smaller partner (all
        // rows above j are done) + self pair + negative merged nets here.
        const double demand = L.get(j) + self2 + dneg;
        flag = flag || (Mtj > 0.0 && demand > Mtj);
        gj = 0.0 + (netj - self2);
        if (j + 1 <= B - 1) g += fout + self2;
        step_pairs += row_pairs<B>(act, nz, j);
      }
      if (j + 1 <= B - 1) finish(j + 1, g, Nj1);
      g = gj;
    }
    if (uni) finish(lo, g, Nnext);
    // bins outside [lo, hi+1] take no part in this step: carried over
    if (live) {
#pragma unroll 1
      for (int k = 0; k < B; ++k)
        if (!uni || k < lo || k > hi + 1)
          so[k * kWave + lane] = sb[k * kWave + lane];
    }

    if (flag) {
      // the exact two-pass step (with the limiter) takes over this point
      // for the rest of the call; its state stays the one this step read,
      // in both buffers
      if (live) {
#pragma unroll 1
        for (int k = 0; k < B; ++k) so[k * kWave + lane] = sb[k * kWave + lane];
      }
      a.pending[slot] = a.steps_left - step;
      live = false;
    } else if (live) {
      npairs += step_pairs;
    }
  }
  add_counters(a.counters, npairs);
}


// FP32C: the normalised masses of a lane's bins live in the lane's column
// of an LDS array (lane-private addresses, so no sharing and no barrier)
// rather than in 33 VGPRs: the kernel then fits 128 VGPRs and runs 4 waves
// per SIMD instead of 3 (8.4 KB of LDS per wave at 33 bins, 16 waves per
// CU in 135 KB), which hides more of each pair's dependent chain.
template <int B, int WPB>
struct MassLds {
  float *s;  // this thread's column: bin k at s[k * threads per block]
  __device__ __forceinline__ float get(int k) const {
    return s[k * (kWave * WPB)];
  }
  __device__ __forceinline__ void set(int k, float v) {
    s[k * (kWave * WPB)] = v;
  }
};

// --------------------------------------------------------- FP32C kernel
// Same sweep and double buffering as the FP64 kernel; pair arithmetic in
// FP32, the carried gain and the losses summed in FP64, the update FP64.
template <int B, int WPB>
__global__ void __launch_bounds__(kWave *WPB)
    __attribute__((amdgpu_waves_per_eu(B <= 33 ? 4 : 2))) lane_step_f32c(
        StepArgs a) {
  constexpr int nthr = kWave * WPB;
  __shared__ float mlds[B * nthr];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int slot = blockIdx.x * nthr + tid;
  const int nslots = uniform(a.meta->nslots);
  const int wave_first = uniform(slot & ~(kWave - 1));
  if (wave_first >= nslots) return;
  const int br = wave_bracket(a.meta, wave_first, a.m.nbr);
  // a slot handed to the exact path earlier in the call stays there
  bool live = slot < nslots && a.slot_point[slot] >= 0 && a.pending[slot] == 0;
  const double w = live ? a.wgt[slot] : 0.0;
  const float wf = (float)w;
  const float *__restrict__ Kf = a.m.KfT + (size_t)br * B * B * 2;
  const float *__restrict__ ctf = a.m.ctfT;
  const float *__restrict__ ixf = a.m.invxf;
  const double x1 = ldc(a.m.x);  // x_k = x_1 2^k exactly
  double *const stw0 = a.state + (size_t)wave_first * B;
  double *const stw1 = a.state_alt + (size_t)wave_first * B;
  const double theta = a.m.theta, dt = a.dt;
  unsigned long long npairs = 0;

  for (int step = 0; step < a.nsteps; ++step) {
    // this step reads one buffer and writes the other (opaque per step, see
    // the FP64 kernel)
    double *sb = (step & 1) ? stw1 : stw0;
    double *so = (step & 1) ? stw0 : stw1;
    asm volatile("" : "+s"(sb));
    asm volatile("" : "+s"(so));
    // S1/S2 in FP64; FP32 masses normalised by the FP64 total.
    double Mtot = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const double v = sb[k * kWave + lane];
      Mtot = __dadd_rn(Mtot, live ? ldexp(__dmul_rn(v, x1), k) : 0.0);
    }
    const double thr = theta * Mtot;
    const double inv = Mtot > 0.0 ? 1.0 / Mtot : 0.0;
    uint64_t act = 0;
    MassLds<B, WPB> m;  // active M_k / M_tot (LDS column of this lane)
    m.s = mlds + tid;
    BinsD<B> L;  // losses of bins as the smaller partner (FP64 sums)
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const double v = sb[k * kWave + lane];
      const double Mk = live ? ldexp(__dmul_rn(v, x1), k) : 0.0;
      const bool ak = Mk > 0.0 && Mk >= thr;
      act |= (uint64_t)ak << k;
      m.set(k, ak ? (float)(Mk * inv) : 0.0f);
      L.set(k, 0.0);
    }
    const float tau = (float)(dt * Mtot);
    const uint64_t uni = wave_or64(act);
    const int lo = uniform(uni ? (int)__builtin_ctzll(uni) : 0);
    const int hi = uniform(uni ? 63 - (int)__builtin_clzll(uni) : -1);
    const uint32_t uni_lo = uniform((int)(uint32_t)uni);
    const uint32_t uni_hi = uniform((int)(uint32_t)(uni >> 32));
    bool flag = false;
    unsigned step_pairs = 0;
    // S6 for bin k: FP64 update from the FP64 gain g and losses, written
    // to the other buffer
    auto finish = [&](int k, double g, double Nk) {
      const double Mk = ldexp(__dmul_rn(Nk, x1), k);
      double Mn = Mk + (g - L.get(k)) * Mtot;
      Mn = Mn < 0.0 ? 0.0 : Mn;
      if (live) so[k * kWave + lane] = ldexp(Mn / x1, -k);
    };
    // gain of bin j+1 from its own row (FP64), carried down one row
    double g = 0.0;
    // state of bin j+1, loaded one row ahead of its update (rows run over
    // the union [lo, hi] of the wave's active bins; bins lo..hi+1 change)
    double Nnext = (hi + 1 <= B - 1) ? sb[(hi + 1) * kWave + lane] : 0.0;

    for (int j = hi; j >= lo; --j) {
      const double Nj1 = Nnext;
      Nnext = sb[j * kWave + lane];
      double gj = 0.0;  // gain of bin j from row j
      if (bit_of(uni_lo, uni_hi, j)) {
        double fs = 0.0;     // flux leaving bin j for j+1
        float self2 = 0.0f;  // self-pair mass, bin j -> j+1
        // columns: active in some lane, kernel entry nonzero at some level
        const uint64_t nz = ldc(a.m.nzT + j);
        const uint64_t below_mask =
            ((j == 0) ? 0ull : (~0ull >> (64 - j))) & nz;
        const uint32_t cl = uni_lo & (uint32_t)below_mask;
        const uint32_t ch = uni_hi & (uint32_t)(below_mask >> 32);
        const float mj = m.get(j);
        // guarded log argument below: 2^-126 keeps it positive in lanes
        // where bin j is empty (their pair amounts are zero)
        const float mjg = mj + 0x1p-126f;
        const float tj = (tau * mj) * ldc(ixf + j);  // A = K m_i tj
        // the pressure weight folded into the row factor:
        // tj K = tj K_{l+1} + (tj w) (K_l - K_{l+1})
        const float tjw = tj * wf;
        const bool has_flux = j <= B - 2;
        // slope logs split into exact exponents and mantissa logs (see
        // log2_split: the tail's masses are tiny and their logs large)
        // lam = log2 m_{j+1} - log2(m_j + Sm)
        //     = [log2 m_{j+1} - log2 m_j] - log2(1 + Sm / m_j):
        // the bracket once per row from split logs, the rest per pair as
        // the log of a value in [1, 2) for most pairs
        // (carried as halves: h = lam / 2 = hrow - log2(1 + Sm / m_j) / 2)
        float hrow = 0.0f, imj = 0.0f;
        if (has_flux) {
          int e1, e0;
          float f1, f0;
          log2_split(m.get(j + 1), e1, f1);
          log2_split(mjg, e0, f0);
          hrow = 0.5f * ((float)(e1 - e0) + (f1 - f0));
          imj = __builtin_amdgcn_rcpf(mjg);
          imj = __builtin_fmaf(imj, __builtin_fmaf(-mjg, imj, 1.0f), imj);
        }
        const float *Kj = Kf + (size_t)j * B * 2;  // row j: [i][2]
        const float *cj = ctf + (size_t)j * B * 2;  // row j: [i](c, 2c ln 2)
        double as = 0.0;  // mass arriving in bin j
        // columns in chunks of 8: the chunk's table entries (kernel pair and
        // Courant pair per column) are fetched with a few wide scalar loads
        // before its pairs, instead of one load and wait per pair
#pragma unroll
        for (int i0 = 0; i0 < B - 1; i0 += 8) {
          const uint32_t chunk = (i0 < 32) ? ((cl >> i0) & 0xffu)
                                           : ((ch >> (i0 - 32)) & 0xffu);
          if (!chunk) continue;
          float kk[16], cc[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const bool in = i0 * 2 + u < 2 * (B - 1);  // inside row j
            kk[u] = in ? ldc(Kj + i0 * 2 + u) : 0.0f;
            cc[u] = in ? ldc(cj + i0 * 2 + u) : 0.0f;
          }
          // the chunk's column masses, read from LDS together (one wait
          // for the chunk instead of one per pair)
          float mc[8];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            mc[u] = i0 + u < B - 1 ? m.get(i0 + u) : 0.0f;
#pragma unroll
          for (int i = i0; i < i0 + 8 && i < B - 1; ++i) {
            if (!bit_of(cl, ch, i)) continue;
            const int u = 2 * (i - i0);
            const float tK = __builtin_fmaf(kk[u + 1], tjw, tj * kk[u]);
            const float A = tK * mc[i - i0];
            // x_j / x_i = 2^(j-i) exactly on the doubling grid: the merged
            // mass A + A 2^(j-i), rounded once
            const float p2 = __builtin_bit_cast(float, (127 + j - i) << 23);
            const float Sm = __builtin_fmaf(A, p2, A);
            // every FP32 amount enters its FP64 sums exactly: the sums
            // round only at FP64 precision, and gain and loss of a
            // transfer carry the same value
            const double Ad = (double)A;
            L.set(i, L.get(i) + Ad);
            as += Ad;
            if (has_flux) {
              float h = __builtin_fmaf(
                  __builtin_amdgcn_logf(__builtin_fmaf(Sm, imj, 1.0f)), -0.5f,
                  hrow);
              h = __builtin_amdgcn_fmed3f(h, kHalfLamFloor, kHalfLamCeil);
              const float F =
                  flux_fraction_half_f32(cc[u], cc[u + 1], h) * Sm;
              fs += (double)F;
            }
          }
        }
        // self pair: transfer 2A from bin j to bin j+1 (exact hit, no flux)
        if (j + 1 <= B - 1 && ((nz >> j) & 1ull)) {
          const float *e = Kj + j * 2;
          const float tK = __builtin_fmaf(ldc(e + 1), tjw, tj * ldc(e));
          const float A = 0.5f * (tK * mj);
          self2 = A + A;
        }
        // S5 bound: losses as the smaller partner + self pair + every flux
        // leaving bin j (>= the negative merged nets); FP32 margin.
        const double out = fs + (double)self2;
        flag = flag || (mj > 0.0f && L.get(j) + out > mj * (1.0 - 1e-5));
        // bin j keeps the mass arriving from smaller partners less what it
        // passes on to j+1
        gj = as - out;
        if (j + 1 <= B - 1) g += out;
        step_pairs += row_pairs<B>(act, nz, j);
      }
      if (j + 1 <= B - 1) finish(j + 1, g, Nj1);
      g = gj;
    }
    if (uni) finish(lo, g, Nnext);
    // bins outside [lo, hi+1] take no part in this step: carried over
    if (live) {
#pragma unroll 1
      for (int k = 0; k < B; ++k)
        if (!uni || k < lo || k > hi + 1)
          so[k * kWave + lane] = sb[k * kWave + lane];
    }

    if (flag) {
      // the exact two-pass step (with the limiter) takes over this point
      // for the rest of the call; its state stays the one this step read,
      // in both buffers
      if (live) {
#pragma unroll 1
        for (int k = 0; k < B; ++k) so[k * kWave + lane] = sb[k * kWave + lane];
      }
      a.pending[slot] = a.steps_left - step;
      live = false;
    } else if (live) {
      npairs += step_pairs;
    }
  }
  add_counters(a.counters, npairs);
}

// Exact FP64 steps for lanes the fast kernels handed over.  The compacted
// slot count is known on the device only, so a bounded grid strides over
// the slots (usually none is pending).
__global__ void __launch_bounds__(64) slow_steps(StepArgs a) {
  const int nslots = a.meta->nslots;
  for (int slot = blockIdx.x * blockDim.x + threadIdx.x; slot < nslots;
       slot += gridDim.x * blockDim.x) {
    const int n = a.pending[slot];
    if (n <= 0) continue;
    int br = 0;
    for (int b = 1; b < a.m.nbr; ++b)
      if ((slot & ~(kWave - 1)) >= a.meta->bucket_base[b]) br = b;
    unsigned long long pairs = 0, lim = 0;
    for (int k = 0; k < n; ++k)
      lim += slow_step_f64<kLaneMaxBins>(
          a.m, a.state + state_index(0, slot, a.m.S * a.m.B), kWave,
          a.wgt[slot], br, a.dt, &pairs);
    a.pending[slot] = 0;
    atomicAdd(&a.counters[0], pairs);
    atomicAdd(&a.counters[4], pairs);
    if (lim) atomicAdd(&a.counters[1], lim);
    atomicAdd(&a.counters[2], (unsigned long long)n);
  }
}

template <int B, int WPB>
hipError_t launch_bw(const StepArgs &a, int precision, int max_slots,
                     hipStream_t st) {
  constexpr int threads = kWave * WPB;
  const int blocks = (max_slots + threads - 1) / threads;
  if (blocks == 0) return hipSuccess;
  if (precision == 0)
    hipLaunchKernelGGL((lane_step_f64<B, WPB>), dim3(blocks), dim3(threads),
                       0, st, a);
  else
    hipLaunchKernelGGL((lane_step_f32c<B, WPB>), dim3(blocks),
                       dim3(threads), 0, st, a);
  return hipGetLastError();
}

// Slot capacity is a multiple of kLaneMaxWpb * kWave, so every launched
// thread addresses a slot inside the workspace.
template <int B>
hipError_t launch_b(const StepArgs &a, int precision, int wpb, int max_slots,
                    hipStream_t st) {
  if (wpb == 2) return launch_bw<B, 2>(a, precision, max_slots, st);
  return launch_bw<B, 1>(a, precision, max_slots, st);
}

}  // namespace

hipError_t launch_slow_steps(const StepArgs &a, int max_slots,
                             hipStream_t st) {
  const int blocks = min((max_slots + 63) / 64, 2048);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(slow_steps, dim3(blocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

bool lane_kernel_supported(int B, int S, int s) {
  return S == 1 && s == 1 && (B == 3 || B == 8 || B == 16 || B == 33 ||
                              B == 40);
}

hipError_t launch_lane_step(const StepArgs &a, int precision, int wpb,
                            int max_slots, hipStream_t st) {
  switch (a.m.B) {
    case 3:
      return launch_b<3>(a, precision, wpb, max_slots, st);
    case 8:
      return launch_b<8>(a, precision, wpb, max_slots, st);
    case 16:
      return launch_b<16>(a, precision, wpb, max_slots, st);
    case 33:
      return launch_b<33>(a, precision, wpb, max_slots, st);
    case 40:
      return launch_b<40>(a, precision, wpb, max_slots, st);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fsbm
