// kernels_multi.hip -- one grid point per lane for several particle types:
// the FP32C collision step of points holding two to four species on the
// mass-doubling grid (the liquid, ice, snow and graupel spectra of FSBM,
// 33 bins each, Sec. III), with the species-pair kernels of Sec. VI-A.
//
// Mapping (gfx950):
//  * compaction buckets the cloudy points by pressure bracket and by the
//    set of species they can hold during the call (the species present at
//    the point, closed under the product map: a point with ice only can
//    make snow), and pads every bucket to whole waves, so a wave's 64
//    points share one bracket and one species set; a launch per set size
//    NS (1..4) runs the waves of its size, every other wave leaves at once;
//  * the points' state is the tiled structure of arrays of the one-species
//    lane kernels (bin q = species * B + k of the wave's 64 points is one
//    contiguous 512-byte row), double buffered;
//  * the pair loop is wave-uniform: rows j (the larger bin of a pair)
//    descending over the union of the wave's active bins; per row, every
//    ordered pair of the set's species (a at the smaller bin i < j, b at
//    j), columns i unrolled; kernel entries of the ordered species pair
//    (transposed to [j][i]) and Courant numbers are scalar loads;
//  * the normalised masses of the point's NS x B bins stay in VGPRs (column
//    bins by static index, the row bin by a wave-uniform index);
//  * on the doubling grid a pair i < j lands in bin j of its product
//    species P with Courant number 2^(i-j), the same-bin pairs land exactly
//    in bin j+1; so bin k of every species is final once rows > k, row k
//    and row k-1 are done, and the descending sweep writes bin j+1 of every
//    species right after row j, carrying a few FP64 sums per species;
//  * the losses of a bin as the smaller partner (rows above it) are not
//    held per bin: when the sweep reaches row k it recomputes each such
//    pair's collided mass with the operation sequence the gain side used,
//    so both sides of every transfer carry the same FP32 value (each pair
//    costs about eight more instructions instead of S x B FP64 registers).
// Arithmetic as in the one-species FP32C lane kernel: masses normalised by
// the point's FP64 total, pair amounts and flux fraction in FP32, every
// transfer's FP32 amount summed per bin in FP64, FP64 totals and update.  A
// lane whose conservative bound on a bin's demand exceeds half the bin's
// mass (the positivity limiter may fire, or the bin drains so far that
// FP32's relative error of the demand would dominate what remains) leaves
// the point, untouched by that step, pending; the one-point-per-wave
// kernel's FP64 mode takes it through the rest of the call.
#include <float.h>

#include "device_common.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

// FP32 bin array with wave-uniform dynamic reads (see BinsD).
template <int N>
struct VecF {
  typedef float type __attribute__((ext_vector_type(N)));
};

template <int B>
struct BinsF {
  static_assert(B >= 2 && B <= 48, "BinsF holds 2..48 bins");
  static constexpr int N0 = B < 16 ? B : 16;
  static constexpr int N1 = B > 16 ? (B - 16 < 16 ? B - 16 : 16) : 1;
  static constexpr int N2 = B > 32 ? B - 32 : 1;
  typename VecF<N0>::type c0;
  typename VecF<N1>::type c1;
  typename VecF<N2>::type c2;
  __device__ __forceinline__ float get(int k) const {
    return (k < 16) ? c0[k] : ((k < 32) ? c1[k - 16] : c2[k - 32]);
  }
  __device__ __forceinline__ void set(int k, float v) {
    if (k < 16)
      c0[k] = v;
    else if (k < 32)
      c1[k - 16] = v;
    else
      c2[k - 32] = v;
  }
};

__device__ __forceinline__ bool bit64(uint64_t v, int k) {
  return ((v >> k) & 1ull) != 0;
}

// Bucket of the slot (the compaction pads every bucket to whole waves).
__device__ __forceinline__ int slot_bucket(const CompactMeta *meta, int slot,
                                           int nbuckets) {
  int bk = 0;
  for (int b = 1; b < nbuckets; ++b)
    if (slot >= meta->bucket_base[b]) bk = b;
  return bk;
}

// Select v[t] for a wave-uniform t < NS (a short chain of selects).
template <int NS, typename T>
__device__ __forceinline__ T pick(const T (&v)[NS], int t) {
  T r = v[0];
#pragma unroll
  for (int u = 1; u < NS; ++u)
    if (t == u) r = v[u];
  return r;
}

template <int NS, typename T>
__device__ __forceinline__ void add_at(T (&v)[NS], int t, T x) {
#pragma unroll
  for (int u = 0; u < NS; ++u)
    if (t == u) v[u] += x;
}

// Mass of bin k (wave-uniform) of species slot t (wave-uniform).
template <int B, int NS>
__device__ __forceinline__ float mass_dyn(const BinsF<B> (&mf)[NS], int t,
                                          int k) {
  float r = mf[0].get(k);
#pragma unroll
  for (int u = 1; u < NS; ++u)
    if (t == u) r = mf[u].get(k);
  return r;
}

// Mass of bin i (static) of species slot t (wave-uniform).
template <int B, int NS>
__device__ __forceinline__ float mass_at(const BinsF<B> (&mf)[NS], int t,
                                         int i) {
  float r = mf[0].get(i);
#pragma unroll
  for (int u = 1; u < NS; ++u)
    if (t == u) r = mf[u].get(i);
  return r;
}

// The pairs (a at columns i < j, b at j) of one ordered species pair, the
// merged mass landing in bin j of species P.  A = tK m_i with the row
// factors tj = tau m_j / x_j and tjw = tj w, tK = tjw (K_l - K_{l+1}) +
// tj K_{l+1}.  OWN (P == b): the target is bin (b, j) itself, which keeps
// the larger partner's collided mass; the flux slope takes the one-species
// lane kernel's form, a per-row bracket (q0) less half the log of
// 1 + Sm / m_j (q1 = 1 / m_j).  Otherwise (b, j) loses its collided mass
// A 2^(j-i) to (P, j), and the slope comes from split logs of P's bins
// (q0 = m_{P,j}, q1 and qe: split log of m_{P,j+1}).  Sums: mass arriving
// in (P, j), mass leaving (b, j), flux leaving (P, j) for (P, j+1), and the
// negative parts of (b, j)'s merged nets A - F (OWN).
template <bool OWN, int B, int NS>
__device__ __forceinline__ void pair_block(
    const BinsF<B> (&mf)[NS], int ta, uint32_t cl, uint32_t ch, int j,
    bool has_flux, float tj, float tjw, const float *Kj, const float *cj,
    float q0, float q1, int qe, double &s_as, double &s_lb, double &s_fo,
    double &s_dn) {
#pragma unroll
  for (int i0 = 0; i0 < B - 1; i0 += 8) {
    const uint32_t chunk = (i0 < 32) ? ((cl >> i0) & 0xffu)
                                     : ((ch >> (i0 - 32)) & 0xffu);
    if (!chunk) continue;
    float kk[16], cc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const bool in = i0 * 2 + u < 2 * (B - 1);
      kk[u] = in ? ldc(Kj + i0 * 2 + u) : 0.0f;
      cc[u] = in ? ldc(cj + i0 * 2 + u) : 0.0f;
    }
#pragma unroll
    for (int i = i0; i < i0 + 8 && i < B - 1; ++i) {
      if (!(((i < 32) ? (cl >> i) : (ch >> (i - 32))) & 1u)) continue;
      const int u = 2 * (i - i0);
      const float tK = __builtin_fmaf(kk[u + 1], tjw, tj * kk[u]);
      const float A = tK * mass_at(mf, ta, i);
      // x_j / x_i = 2^(j-i) exactly: the larger partner's collided mass is
      // an exact scaling of A, the merged mass is rounded once
      const float p2 = __builtin_bit_cast(float, (127 + j - i) << 23);
      const float Sm = __builtin_fmaf(A, p2, A);
      s_as += (double)A;
      if (!OWN) {
        const double Bd = (double)(A * p2);
        s_as += Bd;
        s_lb += Bd;
      }
      if (has_flux) {
        float h;
        if (OWN) {
          h = __builtin_fmaf(
              __builtin_amdgcn_logf(__builtin_fmaf(Sm, q1, 1.0f)), -0.5f, q0);
        } else {
          const float den = __builtin_fmaxf(q0 + Sm, 0x1p-120f);
          int ed;
          float fd;
          log2_split(den, ed, fd);
          h = 0.5f * ((float)(qe - ed) + (q1 - fd));
        }
        h = __builtin_amdgcn_fmed3f(h, kHalfLamFloor, kHalfLamCeil);
        const float F = flux_fraction_half_f32(cc[u], cc[u + 1], h) * Sm;
        s_fo += (double)F;
        if (OWN) s_dn += (double)__builtin_fmaxf(F - A, 0.0f);
      }
    }
  }
}

// FP32C steps run only while no bin's demand (losses and negative merged
// nets) exceeds this fraction of its mass: the positivity limiter needs
// more than all of it, and a bin drained this far would carry FP32's
// relative error of the demand into the little it keeps, step after step
constexpr double kDrainMulti = 0.5;

template <int NS>
struct MultiOcc {
  static constexpr int waves = NS <= 1 ? 4 : (NS == 2 ? 3 : 2);
};

template <int B, int NS>
__global__ void __launch_bounds__(kWave)
    __attribute__((amdgpu_waves_per_eu(MultiOcc<NS>::waves)))
    lane_multi_f32c(StepArgs a) {
  const int tid = threadIdx.x;
  const int lane = tid;
  const int slot = blockIdx.x * kWave + tid;
  const int nslots = uniform(a.meta->nslots);
  const int wave_first = uniform(slot & ~(kWave - 1));
  if (wave_first >= nslots) return;
  const int S = a.m.S, SB = S * B, nmask = a.m.nmask;
  const int bk = uniform(slot_bucket(a.meta, wave_first, a.m.nbr * nmask));
  const int br = bk / nmask;
  const unsigned set = (unsigned)(bk - br * nmask);
  if (__builtin_popcount(set) != NS) return;  // another launch's wave
  // the set's species in ascending order
  int sp[NS];
  {
    unsigned r = set;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      sp[t] = __builtin_ctz(r);
      r &= r - 1u;
    }
  }
  bool live = slot < nslots && a.slot_point[slot] >= 0 && a.pending[slot] == 0;
  const double w = live ? a.wgt[slot] : 0.0;
  const float wf = (float)w;
  const float *__restrict__ ctf = a.m.ctfT;
  const float *__restrict__ ixf = a.m.invxf;
  const double x1 = ldc(a.m.x);  // x_k = x_1 2^k exactly
  double *const stw0 = a.state + (size_t)wave_first * SB;
  double *const stw1 = a.state_alt + (size_t)wave_first * SB;
  const double theta = a.m.theta, dt = a.dt;
  const size_t kstride = (size_t)a.m.nbr * B * B * 2;  // per ordered pair
  const float *__restrict__ Kbr = a.m.KfO + (size_t)br * B * B * 2;
  unsigned long long npairs = 0;

  for (int step = 0; step < a.nsteps; ++step) {
    double *sb = (step & 1) ? stw1 : stw0;  // read
    double *so = (step & 1) ? stw0 : stw1;  // written
    asm volatile("" : "+s"(sb));
    asm volatile("" : "+s"(so));
    // species outside the set hold nothing for the whole call: copied once
    // (both buffers then hold them)
    if (live && step == 0 && a.first_launch) {
      for (int s = 0; s < S; ++s) {
        if ((set >> s) & 1u) continue;
        for (int k = 0; k < B; ++k)
          so[(s * B + k) * kWave + lane] = sb[(s * B + k) * kWave + lane];
      }
    }
    // per species slot: scalar base of its rows in both buffers, opaque per
    // step (bin k of this lane's point at base[k * 64 + lane], one scalar
    // base and immediate offsets, no per-bin 64-bit lane addresses)
    double *sbt[NS], *sot[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      sbt[t] = sb + (size_t)sp[t] * B * kWave;
      sot[t] = so + (size_t)sp[t] * B * kWave;
      asm volatile("" : "+s"(sbt[t]));
      asm volatile("" : "+s"(sot[t]));
    }
    // S1/S2: FP64 total (species ascending, then bins), activity, FP32
    // masses normalised by the total.  Lanes that do not step (padding,
    // points handed to the exact path) see zero masses; the loads stay
    // unconditional (a bit mask, not a branch per bin).
    const unsigned long long keep = live ? ~0ull : 0ull;
    auto mass_of = [&](double v, int k) {
      return __longlong_as_double(
          __double_as_longlong(ldexp(__dmul_rn(v, x1), k)) & keep);
    };
    double Mtot = 0.0;
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int k = 0; k < B; ++k)
        Mtot = __dadd_rn(Mtot, mass_of(sbt[t][k * kWave + lane], k));
    const double thr = theta * Mtot;
    const double inv = Mtot > 0.0 ? 1.0 / Mtot : 0.0;
    BinsF<B> mf[NS];
    uint64_t act[NS], uni[NS];
    uint64_t U = 0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      // read the bins again rather than keep NS x B FP64 values live
      double *sr = sbt[t];
      asm volatile("" : "+s"(sr));
      act[t] = 0;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const double Mk = mass_of(sr[k * kWave + lane], k);
        const bool ak = Mk > 0.0 && Mk >= thr;
        act[t] |= (uint64_t)ak << k;
        mf[t].set(k, ak ? (float)(Mk * inv) : 0.0f);
      }
      const uint64_t o = wave_or64(act[t]);
      uni[t] = ((uint64_t)(uint32_t)uniform((int)(uint32_t)(o >> 32)) << 32) |
               (uint32_t)uniform((int)(uint32_t)o);
      U |= uni[t];
    }
    const float tau = (float)(dt * Mtot);
    const int lo = uniform(U ? (int)__builtin_ctzll(U) : 0);
    const int hi = uniform(U ? 63 - (int)__builtin_clzll(U) : -1);
    bool flag = false;
    unsigned step_pairs = 0;
    // S6 for bin k of species slot t: FP64 update into the other buffer
    auto finish = [&](int t, int k, double net) {
      const double Nk = sbt[t][k * kWave + lane];
      const double Mk = ldexp(__dmul_rn(Nk, x1), k);
      double Mn = Mk + net * Mtot;
      Mn = Mn < 0.0 ? 0.0 : Mn;
      if (live) sot[t][k * kWave + lane] = ldexp(Mn / x1, -k);
    };
    // net change of bin j+1 of each species slot gathered so far: its own
    // row's (mass arriving, less losses as larger partner and in same-bin
    // pairs, less flux out, less losses as smaller partner), then row j's
    // flux and same-bin merges into it
    double ncar[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) ncar[t] = 0.0;

    for (int j = hi; j >= lo; --j) {
      const bool has_flux = j <= B - 2;
      const uint64_t below = (j == 0) ? 0ull : (~0ull >> (64 - j));
      // per species slot, bin j: mass arriving (as), losses as larger
      // partner and in same-bin pairs (lx), flux out (fo), losses as
      // smaller partner (lsm), negative merged nets (dn)
      double as[NS], lx[NS], fo[NS], lsm[NS], dn[NS];
      float mj[NS], tjr[NS], tjwr[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        as[t] = lx[t] = fo[t] = lsm[t] = dn[t] = 0.0;
        mj[t] = mf[t].get(j);
        tjr[t] = (tau * mj[t]) * ldc(ixf + j);
        tjwr[t] = tjr[t] * wf;
      }
      // (1) losses of bins (t, j) as the smaller partner of the rows
      // above: the gain side's collided masses, recomputed identically
      for (int t = 0; t < NS; ++t) {
        if (!bit64(uni[t], j)) continue;
        const float mt = pick(mj, t);
        double acc = 0.0;
        for (int jp = j + 1; jp <= hi; ++jp) {
          for (int tb = 0; tb < NS; ++tb) {
            if (!bit64(uni[tb], jp)) continue;
            const int ob = sp[t] * S + sp[tb];
            if (!((ldc(a.m.nzO + (size_t)ob * B + jp) >> j) & 1ull)) continue;
            const float mb = mass_dyn(mf, tb, jp);
            const float tj = (tau * mb) * ldc(ixf + jp);
            const float tjw = tj * wf;
            const float *e =
                Kbr + (size_t)ob * kstride + ((size_t)jp * B + j) * 2;
            const float tK = __builtin_fmaf(ldc(e + 1), tjw, tj * ldc(e));
            acc += (double)(tK * mt);
          }
        }
        add_at(lsm, t, acc);
      }
      // (2) pairs (a at i < j, b at j) of every ordered species pair:
      // target bin j of P = product(a, b)
      for (int tb = 0; tb < NS; ++tb) {
        if (!bit64(uni[tb], j)) continue;
        const float tj = pick(tjr, tb), tjw = pick(tjwr, tb);
        for (int ta = 0; ta < NS; ++ta) {
          const int ob = sp[ta] * S + sp[tb];
          const uint64_t nz = ldc(a.m.nzO + (size_t)ob * B + j);
          const uint64_t cols = uni[ta] & nz & below;
          if (!cols) continue;
          const uint32_t cl = (uint32_t)cols, ch = (uint32_t)(cols >> 32);
          const int P = ldc(a.m.product + ob);
          int tP = 0;
#pragma unroll
          for (int u = 0; u < NS; ++u)
            if (sp[u] == P) tP = u;
          const float *Kj = Kbr + (size_t)ob * kstride + (size_t)j * B * 2;
          const float *cj = ctf + (size_t)j * B * 2;
          double s_as = 0.0, s_lb = 0.0, s_fo = 0.0, s_dn = 0.0;
          const float mq = pick(mj, tP);
          if (tP == tb) {
            // slope bracket of the row from split logs of bins j+1 and j
            float hr = 0.0f, im = 0.0f;
            if (has_flux) {
              const float mqg = mq + 0x1p-126f;
              int e1, e0;
              float f1, f0;
              log2_split(mass_dyn(mf, tP, j + 1), e1, f1);
              log2_split(mqg, e0, f0);
              hr = 0.5f * ((float)(e1 - e0) + (f1 - f0));
              const float r = __builtin_amdgcn_rcpf(mqg);
              im = __builtin_fmaf(r, __builtin_fmaf(-mqg, r, 1.0f), r);
            }
            pair_block<true>(mf, ta, cl, ch, j, has_flux, tj, tjw, Kj, cj, hr,
                             im, 0, s_as, s_lb, s_fo, s_dn);
          } else {
            int e1 = 0;
            float f1 = 0.0f;
            if (has_flux) log2_split(mass_dyn(mf, tP, j + 1), e1, f1);
            pair_block<false>(mf, ta, cl, ch, j, has_flux, tj, tjw, Kj, cj,
                              mq, f1, e1, s_as, s_lb, s_fo, s_dn);
          }
          add_at(as, tP, s_as);
          add_at(fo, tP, s_fo);
          add_at(lx, tb, s_lb);
          add_at(dn, tb, s_dn);
          if (bit64(pick(act, tb), j))
            step_pairs += (unsigned)__popcll(pick(act, ta) & nz & below);
        }
      }
      // (3) same-bin pairs (a at j, b at j, a <= b): land exactly in bin
      // j+1 of P, no flux
      if (j + 1 <= B - 1) {
        for (int tb = 0; tb < NS; ++tb) {
          if (!bit64(uni[tb], j)) continue;
          for (int ta = 0; ta <= tb; ++ta) {
            if (!bit64(uni[ta], j)) continue;
            const int ob = sp[ta] * S + sp[tb];
            if (!((ldc(a.m.nzO + (size_t)ob * B + j) >> j) & 1ull)) continue;
            const float *e =
                Kbr + (size_t)ob * kstride + ((size_t)j * B + j) * 2;
            const float tK = __builtin_fmaf(ldc(e + 1), pick(tjwr, tb),
                                            pick(tjr, tb) * ldc(e));
            float A = tK * pick(mj, ta);
            if (ta == tb) A = 0.5f * A;
            const int P = ldc(a.m.product + ob);
            int tP = 0;
#pragma unroll
            for (int u = 0; u < NS; ++u)
              if (sp[u] == P) tP = u;
            const double Ad = (double)A;
            add_at(lx, ta, Ad);
            add_at(lx, tb, Ad);
            add_at(ncar, tP, Ad + Ad);
            if (bit64(pick(act, ta), j) && bit64(pick(act, tb), j))
              step_pairs += 1u;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        // (4) S5 demand of bin (t, j): losses as smaller and larger
        // partner and in same-bin pairs, negative merged nets; past half
        // the bin's mass the point leaves the FP32C steps
        const double D = (lsm[t] + lx[t]) + dn[t];
        flag = flag || (mj[t] > 0.0f && D > kDrainMulti * (double)mj[t]);
        // (5) bin j+1 is final: update it; start bin j's net
        if (j + 1 <= B - 1) finish(t, j + 1, ncar[t] + fo[t]);
        ncar[t] = ((as[t] - lx[t]) - fo[t]) - lsm[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t)
      if (U) finish(t, lo, ncar[t]);
    // bins of the set's species outside [lo, hi+1] take no part: carried
    if (live) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
#pragma unroll 1
        for (int k = 0; k < B; ++k)
          if (!U || k < lo || k > hi + 1)
            sot[t][k * kWave + lane] = sbt[t][k * kWave + lane];
      }
    }
    if (flag) {
      // the exact two-pass step (with the limiter) takes over this point
      // for the rest of the call; its state stays the one this step read,
      // in both buffers
      if (live) {
#pragma unroll 1
        for (int q = 0; q < SB; ++q) so[q * kWave + lane] = sb[q * kWave + lane];
      }
      a.pending[slot] = a.steps_left - step;
      live = false;
    } else if (live) {
      npairs += step_pairs;
    }
  }
  npairs = wave_sum_u64(npairs);
  if (lane == 0 && npairs) atomicAdd(&a.counters[0], npairs);
}

template <int B>
hipError_t launch_multi_b(const StepArgs &a, int max_slots, hipStream_t st) {
  const int blocks = (max_slots + kWave - 1) / kWave;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((lane_multi_f32c<B, 1>), dim3(blocks), dim3(kWave), 0,
                     st, a);
  hipLaunchKernelGGL((lane_multi_f32c<B, 2>), dim3(blocks), dim3(kWave), 0,
                     st, a);
  if (a.m.S >= 3)
    hipLaunchKernelGGL((lane_multi_f32c<B, 3>), dim3(blocks), dim3(kWave), 0,
                       st, a);
  if (a.m.S >= 4)
    hipLaunchKernelGGL((lane_multi_f32c<B, 4>), dim3(blocks), dim3(kWave), 0,
                       st, a);
  return hipGetLastError();
}

}  // namespace

bool multi_kernel_supported(int B, int S, int s, int nbr) {
  return S >= 2 && S <= kMultiMaxSpecies && s == 1 && B == 33 &&
         nbr * (1 << S) <= kMaxBuckets;
}

hipError_t launch_multi_step(const StepArgs &a, int max_slots,
                             hipStream_t st) {
  if (a.m.B == 33) return launch_multi_b<33>(a, max_slots, st);
  return hipErrorInvalidValue;
}

}  // namespace fsbm
