// kernels_wave.hip -- one grid point per wave: the collision step for any
// species set and any bin grid (several particle types with their pair
// kernels and product rules, refined grids up to hundreds of bins; Sec. III:
// "33 bins ... extendable to a few hundreds"), over one or several grids in
// one persistent launch.
//
// Mapping (gfx950):
//  * a wave (one 64-thread block) owns one point at a time and loops over
//    the compacted points of every grid of the launch (persistent grid);
//  * the point's bins are spread over the lanes by a load-balanced schedule
//    built at create time; each lane owns up to kMaxOwn bins and keeps their
//    accumulators in registers;
//  * the point's masses, numbers and log-masses sit in LDS for all lanes;
//  * gains: the owner of bin (P,k) walks the precomputed list of pairs whose
//    merged mass lands in (P,k) and evaluates each such pair once (collided
//    masses, exponential-profile flux fraction); the flux leaving (P,k) for
//    (P,k+1) is handed over through LDS;
//  * losses: the owner of a source bin recomputes the same collided mass of
//    each of its pairs (the identical operation sequence, hence the identical
//    value), so every transfer is applied symmetrically and no cross-lane
//    accumulation or atomic is needed; results do not depend on timing;
//  * a conservative over-demand bound per bin (losses + outgoing flux)
//    hands the rare point that may need the positivity limiter to the exact
//    FP64 path (wave_slow, global scratch).
// FP64 mode: the method in FP64 with FP64 sums.  FP32C mode: normalised
// masses, FP32 pair arithmetic, compensated FP32 sums (TwoSum error
// capture), FP64 totals and FP64 update.
#include <float.h>

#include <type_traits>

#include "device_common.hpp"
#include "slow_path.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

struct AccF64 {
  double v;
  __device__ __forceinline__ void zero() { v = 0.0; }
  __device__ __forceinline__ void add(double x) { v += x; }
  __device__ __forceinline__ double val() const { return v; }
};

struct AccF32 {
  float s, c;
  __device__ __forceinline__ void zero() { s = c = 0.0f; }
  __device__ __forceinline__ void add(float x) { comp_add(s, c, x); }
  __device__ __forceinline__ double val() const {
    return (double)s + (double)c;
  }
};

__device__ __forceinline__ double wave_sum_f64(double v) {
  // butterfly: every lane ends with the same value (each stage adds the
  // same two numbers in every lane)
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ int species_pair(int S, int a, int b) {
  return a * S - (a * (a - 1)) / 2 + (b - a);
}

struct PairIdx {
  int i, j, a, b;
};

__device__ __forceinline__ PairIdx unpack(unsigned e) {
  PairIdx p;
  p.i = (int)(e & 511u);
  p.j = (int)((e >> 9) & 511u);
  p.a = (int)((e >> 18) & 7u);
  p.b = (int)((e >> 21) & 7u);
  return p;
}

// Collided amounts of one pair in FP64: A leaves (a,i), Bm leaves (b,j).
__device__ __forceinline__ void amounts_f64(const DevModel &m, int br,
                                            double w, double dt,
                                            const double *Nv,
                                            const PairIdx &p, double &A,
                                            double &Bm) {
  const int B = m.B;
  const int ab = species_pair(m.S, p.a, p.b);
  const double *e =
      m.Kd + ((((size_t)ab * m.nbr + br) * B + p.i) * B + p.j) * 2;
  const double K = fma(e[1], w, e[0]);
  double C = dt * K * Nv[p.a * B + p.i] * Nv[p.b * B + p.j];
  if (p.a == p.b && p.i == p.j) C *= 0.5;
  A = C * m.x[p.i];
  Bm = C * m.x[p.j];
}

// The same in FP32 on numbers normalised by the point's mass (tau = dt
// M_tot): amounts come out normalised by M_tot.
__device__ __forceinline__ void amounts_f32(const DevModel &m, int br,
                                            float wf, float tau,
                                            const float *nv,
                                            const PairIdx &p, float &A,
                                            float &Bm) {
  const int B = m.B;
  const int ab = species_pair(m.S, p.a, p.b);
  const float *e =
      m.Kf + ((((size_t)ab * m.nbr + br) * B + p.i) * B + p.j) * 2;
  const float K = __builtin_fmaf(e[1], wf, e[0]);
  float C = ((tau * K) * nv[p.a * B + p.i]) * nv[p.b * B + p.j];
  if (p.a == p.b && p.i == p.j) C *= 0.5f;
  A = C * m.xf[p.i];
  Bm = C * m.xf[p.j];
}

// One step of one point by one wave.  Returns false (state untouched) if
// the over-demand bound fired and the exact path must take the step.
template <bool F32>
__device__ bool point_step(const DevModel &m, double *st, double w, int br,
                           double dt, unsigned char *lds,
                           unsigned long long &npairs) {
  typedef typename std::conditional<F32, AccF32, AccF64>::type Acc;
  const int lane = threadIdx.x;
  const int B = m.B, SB = m.S * m.B;
  // LDS: FP64 mode Mt, Nv, lnM, fout (doubles); FP32 mode m, n, lm, fs, fc
  double *Mt_l = (double *)lds;
  double *Nv_l = Mt_l + SB;
  double *ln_l = Nv_l + SB;
  double *fo_l = ln_l + SB;
  float *m_l = (float *)lds;
  float *n_l = m_l + SB;
  float *lm_l = n_l + SB;
  float *fs_l = lm_l + SB;
  float *fc_l = fs_l + SB;
  const short *own = m.own + lane * kMaxOwn;

  // S1/S2: owned bins, FP64 total, activity
  double Mown[kMaxOwn];
  double part = 0.0;
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    Mown[o] = 0.0;
    if (q >= 0) {
      Mown[o] = st[q] * m.x[q % B];
      part += Mown[o];
    }
  }
  const double Mtot = wave_sum_f64(part);
  const double thr = m.theta * Mtot;
  const double inv = Mtot > 0.0 ? 1.0 / Mtot : 0.0;
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    const double Mq = Mown[o];
    const bool act = Mq > 0.0 && Mq >= thr;
    const double Mt = act ? Mq : 0.0;
    if constexpr (F32) {
      const float mq = (float)(Mt * inv);
      m_l[q] = mq;
      n_l[q] = (float)((act ? st[q] : 0.0) * inv);
      lm_l[q] = __builtin_amdgcn_logf(mq);
    } else {
      Mt_l[q] = Mt;
      Nv_l[q] = act ? st[q] : 0.0;
      ln_l[q] = log(Mt);
    }
  }
  __syncthreads();
  const float wf = (float)w;
  const float tau = (float)(dt * Mtot);

  // S3/S4 gains: pairs landing in each owned bin, flux to the next bin
  Acc gain[kMaxOwn], fout[kMaxOwn], loss[kMaxOwn];
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    gain[o].zero();
    fout[o].zero();
    loss[o].zero();
  }
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    const int k = q % B;
    const bool has_flux = k <= B - 2;
    const int e0 = m.tgt_off[q], e1 = m.tgt_off[q + 1];
    for (int e = e0; e < e1; ++e) {
      const unsigned ent = m.tgt_ent[e];
      const PairIdx p = unpack(ent);
      const int qa = p.a * B + p.i, qb = p.b * B + p.j;
      if constexpr (F32) {
        if (m_l[qa] == 0.0f || m_l[qb] == 0.0f) continue;
        float A, Bm;
        amounts_f32(m, br, wf, tau, n_l, p, A, Bm);
        float F = 0.0f;
        if (has_flux) {
          const float Sm = A + Bm;
          const float den = __builtin_fmaxf(m_l[q] + Sm, 0x1p-120f);
          float lam = lm_l[q + 1] - __builtin_amdgcn_logf(den);
          lam = __builtin_amdgcn_fmed3f(lam, kLamFloor, kLamCeil);
          const float c = m.ctf[p.i * B + p.j];
          F = flux_fraction_f32(c, c * kLn2f, lam) * Sm;
        }
        if (!(ent & kEntTA)) gain[o].add(A);
        if (!(ent & kEntTB)) gain[o].add(Bm);
        gain[o].add(-F);
        fout[o].add(F);
      } else {
        if (Mt_l[qa] == 0.0 || Mt_l[qb] == 0.0) continue;
        double A, Bm;
        amounts_f64(m, br, w, dt, Nv_l, p, A, Bm);
        double F = 0.0;
        if (has_flux) {
          const double Sm = A + Bm;
          const double den = fmax(Mt_l[q] + Sm, DBL_MIN);
          const double x1 = fmax(ln_l[q + 1] - log(den), kX1Floor);
          F = flux_fraction_f64(m.ct[p.i * B + p.j], x1) * Sm;
        }
        // the pair's combined contribution to its target in one rounding
        // (a target that is also a source keeps the other source's mass)
        const double keep =
            (ent & kEntTA) ? Bm : ((ent & kEntTB) ? A : A + Bm);
        gain[o].add(keep - F);
        fout[o].add(F);
      }
      ++npairs;
    }
  }
  // hand the flux of bin (P,k) to the owner of (P,k+1)
  __syncthreads();
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    if constexpr (F32) {
      fs_l[q] = fout[o].s;
      fc_l[q] = fout[o].c;
    } else {
      fo_l[q] = fout[o].v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0 || q % B == 0) continue;
    if constexpr (F32) {
      gain[o].add(fs_l[q - 1]);
      gain[o].add(fc_l[q - 1]);
    } else {
      gain[o].add(fo_l[q - 1]);
    }
  }

  // losses: the same collided amounts, seen from the source bins
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    bool active;
    if constexpr (F32)
      active = m_l[q] != 0.0f;
    else
      active = Mt_l[q] != 0.0;
    if (!active) continue;
    const int e0 = m.loss_off[q], e1 = m.loss_off[q + 1];
    for (int e = e0; e < e1; ++e) {
      const unsigned ent = m.loss_ent[e];
      const PairIdx p = unpack(ent);
      const int partner = (ent & kEntSideB) ? p.a * B + p.i : p.b * B + p.j;
      if constexpr (F32) {
        if (m_l[partner] == 0.0f) continue;
        float A, Bm;
        amounts_f32(m, br, wf, tau, n_l, p, A, Bm);
        if (ent & kEntSelf) {
          loss[o].add(A);
          loss[o].add(Bm);
        } else {
          loss[o].add((ent & kEntSideB) ? Bm : A);
        }
      } else {
        if (Mt_l[partner] == 0.0) continue;
        double A, Bm;
        amounts_f64(m, br, w, dt, Nv_l, p, A, Bm);
        if (ent & kEntSelf) {
          loss[o].add(A);
          loss[o].add(Bm);
        } else {
          loss[o].add((ent & kEntSideB) ? Bm : A);
        }
      }
    }
  }

  // S5 bound: demand <= losses + outgoing flux (the merged net of a bin
  // that is also its pair's target is A - F >= -F)
  bool flag = false;
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    double Mq;
    if constexpr (F32)
      Mq = (double)m_l[q];
    else
      Mq = Mt_l[q];
    if (Mq == 0.0) continue;
    const double demand = loss[o].val() + fout[o].val();
    flag = flag || demand > Mq * (F32 ? (1.0 - 1e-5) : (1.0 - 1e-9));
  }
  const bool any_flag = __any(flag);
  __syncthreads();  // LDS is rewritten by the next step
  if (any_flag) return false;

  // S6: FP64 update of the owned bins
#pragma unroll
  for (int o = 0; o < kMaxOwn; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    double net = gain[o].val() - loss[o].val();
    if constexpr (F32) net *= Mtot;
    double Mn = Mown[o] + net;
    Mn = Mn < 0.0 ? 0.0 : Mn;
    st[q] = Mn / m.x[q % B];
  }
  return true;
}

template <bool F32>
__global__ void __launch_bounds__(kWave) wave_step(WaveArgs a) {
  extern __shared__ unsigned char lds[];
  unsigned long long npairs = 0;
  for (int g = 0; g < a.ngrids; ++g) {
    const WaveGrid &G = a.g[g];
    const DevModel &m = G.m;
    const int SB = m.S * m.B;
    const int nslots = G.meta->nslots;
    for (int slot = blockIdx.x; slot < nslots; slot += gridDim.x) {
      const int pt = G.slot_point[slot];
      // padding, or a point handed to the exact path earlier in the call
      if (pt < 0 || G.pending[slot] != 0) continue;
      int br = 0;
      for (int b = 1; b < m.nbr; ++b)
        if (slot >= G.meta->bucket_base[b]) br = b;
      const double w = G.wgt[slot];
      double *st = G.state + (size_t)slot * SB;
      for (int step = 0; step < a.nsteps; ++step) {
        unsigned long long pc = 0;
        const bool ok = point_step<F32>(m, st, w, br, a.dt, lds, pc);
        if (!ok) {
          if (threadIdx.x == 0) G.pending[slot] = a.steps_left - step;
          break;
        }
        npairs += pc;
      }
    }
  }
  npairs = wave_sum_u64(npairs);
  if (threadIdx.x == 0 && npairs) atomicAdd(&a.counters[0], npairs);
}

// Exact FP64 steps for points the fast kernel handed over.
__global__ void __launch_bounds__(64) wave_slow(WaveArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double *work = a.scratch + (size_t)t * 7 * a.scratch_sb;
  unsigned long long pairs = 0, lim = 0, fb = 0;
  for (int g = 0; g < a.ngrids; ++g) {
    const WaveGrid &G = a.g[g];
    const int SB = G.m.S * G.m.B;
    const int nslots = G.meta->nslots;
    for (int slot = t; slot < nslots; slot += kSlowThreads) {
      const int n = G.pending[slot];
      if (n <= 0) continue;
      int br = 0;
      for (int b = 1; b < G.m.nbr; ++b)
        if (slot >= G.meta->bucket_base[b]) br = b;
      for (int k = 0; k < n; ++k)
        lim += slow_step_core(G.m, G.state + (size_t)slot * SB, 1,
                              G.wgt[slot], br, a.dt, &pairs, work);
      fb += (unsigned long long)n;
      G.pending[slot] = 0;
    }
  }
  if (pairs) atomicAdd(&a.counters[0], pairs);
  if (lim) atomicAdd(&a.counters[1], lim);
  if (fb) atomicAdd(&a.counters[2], fb);
}

}  // namespace

hipError_t launch_wave_step(const WaveArgs &a, int precision, int blocks,
                            hipStream_t st) {
  int sb = 0;
  for (int g = 0; g < a.ngrids; ++g)
    sb = a.g[g].m.S * a.g[g].m.B > sb ? a.g[g].m.S * a.g[g].m.B : sb;
  const size_t lds = (size_t)sb * 32;
  if (precision == 0)
    hipLaunchKernelGGL(wave_step<false>, dim3(blocks), dim3(kWave), lds, st,
                       a);
  else
    hipLaunchKernelGGL(wave_step<true>, dim3(blocks), dim3(kWave), lds, st,
                       a);
  return hipGetLastError();
}

hipError_t launch_wave_slow(const WaveArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(wave_slow, dim3(kSlowThreads / 64), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace fsbm
