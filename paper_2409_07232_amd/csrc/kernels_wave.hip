// kernels_wave.hip -- one grid point per wave: the collision step for any
// species set and any bin grid (several particle types with their pair
// kernels and product rules; the 33 bins per type of Sec. III refined to a
// few hundred), over one or several grids in one persistent launch.
//
// Mapping (gfx950):
//  * a wave (one 64-thread block) owns one point at a time and loops over
//    the compacted points of every grid of the launch (persistent grid);
//  * the point's bins are spread over the lanes by a load-balanced schedule
//    built at create time; each lane owns up to kMaxOwn bins and keeps their
//    accumulators in registers (builds for at most kOwnSmall or kOwnMid
//    bins per lane run where the schedule fits them: four species at 33
//    bins and two at 66 hold 68 fewer spilled registers at 3 waves per
//    SIMD, FP64 steps 5-6% faster; two species at 132 bins and the mixed
//    batch none at 2 waves, 2-4.5% faster);
//  * the point's masses, numbers and log-masses sit in LDS for all lanes;
//  * each lane walks two precomputed streams of pair entries, interleaved by
//    lane so that entry r of all 64 lanes is one coalesced load and the
//    addresses never depend on loaded data; an entry carries the pair's
//    bins, flags, bin masses, Courant numbers and interpolation pairs;
//  * gains: the owner of bin (P,k) evaluates each pair whose merged mass
//    lands in (P,k) once (collided masses, exponential-profile flux
//    fraction); the flux leaving (P,k) for (P,k+1) is handed over through
//    LDS;
//  * losses: the owner of a source bin recomputes the same collided mass of
//    each of its pairs (the identical operation sequence, hence the identical
//    value), so every transfer is applied symmetrically and no cross-lane
//    accumulation or atomic is needed; results do not depend on timing;
//  * a bin's entries are contiguous in its owner's stream: a running sum in
//    registers is stored to LDS once per bin;
//  * positivity limiter: the first pass also sums each bin's demand (its
//    negative merged nets); if any bin is over-demanded the wave runs the
//    second pass of the method itself, every pair scaled by the smallest
//    sigma = M / D over the bins where the pair's net is negative.
// FP64 mode: the method in FP64 with FP64 sums.  FP32C mode: normalised
// masses, FP32 pair arithmetic, the FP32 amounts summed per bin in FP64
// (each enters its sums exactly, so a transfer leaves and enters with the
// same value), FP64 totals and FP64 update; a point at which the limiter fires
// takes that and every remaining step of the call in FP64 mode (a follow-up
// launch over those points only), since emptying a bin by cancellation
// needs FP64 to stay conservative and positive.
#include <float.h>

#include <type_traits>

#include "device_common.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

// FP32C steps run only while no bin loses more than this fraction of its
// mass in the step (see the S5 check in point_step)
constexpr double kDrainFp32 = 0.5;

struct AccF64 {
  double v;
  __device__ __forceinline__ void zero() { v = 0.0; }
  __device__ __forceinline__ void add(double x) { v += x; }
  __device__ __forceinline__ double val() const { return v; }
};

// FP32 amounts summed in FP64: each amount enters exactly, so the gain and
// the loss side of a transfer carry the same value and the sums round only
// at FP64 precision (an FP64 add issues at the rate of an FP32 one).
struct AccF32 {
  double v;
  __device__ __forceinline__ void zero() { v = 0.0; }
  __device__ __forceinline__ void add(float x) { v += (double)x; }
  __device__ __forceinline__ double val() const { return v; }
};

__device__ __forceinline__ double wave_sum_f64(double v) {
  // butterfly: every lane ends with the same value (each stage adds the
  // same two numbers in every lane)
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// Collided amounts of one stream entry from the numbers na of bin qa and nb
// of bin qb: A leaves qa, Bm leaves qb.
__device__ __forceinline__ void entry_amounts(double K, double dt, double na,
                                              double nb, bool self, double2 x,
                                              double &A, double &Bm) {
  double C = dt * K * na * nb;
  if (self) C *= 0.5;
  A = C * x.x;
  Bm = C * x.y;
}

// The same in FP32 on numbers normalised by the point's mass (tau = dt
// M_tot): amounts come out normalised by M_tot.
__device__ __forceinline__ void entry_amounts(float K, float tau, float na,
                                              float nb, bool self, float2 x,
                                              float &A, float &Bm) {
  float C = ((tau * K) * na) * nb;
  if (self) C *= 0.5f;
  A = C * x.x;
  Bm = C * x.y;
}

// Flux that a pair with merged mass Sm landing in bin qt moves on to qt+1;
// the gain and the loss side call the same function with the same inputs.
// Inlined: as a call it needs every load in flight to land first (the
// batch's operand loads of the next row included); inline, the FP64 steps
// run 2-5% faster with the same results bit for bit.
__device__ __forceinline__ double entry_flux(bool has_flux, const double *Mt,
                                             const double *lnM, int qt,
                                             double c, double Sm) {
  if (!has_flux) return 0.0;
  const double den = fmax(Mt[qt] + Sm, DBL_MIN);
  const double x1 = fmax(lnM[qt + 1] - log_f64(den), kX1Floor);
  return flux_fraction_f64(c, x1) * Sm;
}

// FP32 flux of a gain entry whose merged mass Sm lands in a target with
// normalised mass mq, next bin's split log (le1, lm1): the slope
// log2(m_{k+1} / (m_k + Sm)) from split logs (the exponent difference is
// exact, so the error stays ~1e-7 absolute also where the target is nearly
// empty and Sm dominates), carried as its half.  c = (c, 2 c ln 2).
__device__ __forceinline__ float entry_flux_f32(float mq, int le1, float lm1,
                                                float2 c, float Sm) {
  const float den = __builtin_fmaxf(mq + Sm, 0x1p-120f);
  int ed;
  float fd;
  log2_split(den, ed, fd);
  float h = 0.5f * ((float)(le1 - ed) + (lm1 - fd));
  h = __builtin_amdgcn_fmed3f(h, kHalfLamFloor, kHalfLamCeil);
  return flux_fraction_half_f32(c.x, c.y, h) * Sm;
}

// Limiter scale of a pair: the smallest sigma over the bins where the pair's
// net is negative.  A source bin that does not receive the merged mass has
// net -A (or -Bm); a source bin that does has net Bm - F (or A - F).
template <typename T>
__device__ __forceinline__ T pair_scale(const T *sg, int qa, int qb, bool ta,
                                        bool tb, T A, T Bm, T F) {
  T s = (T)1;
  const bool na = ta ? (Bm - F < (T)0) : (A > (T)0);
  const bool nb = tb ? (A - F < (T)0) : (Bm > (T)0);
  if (na) s = sg[qa] < s ? sg[qa] : s;
  if (nb) s = sg[qb] < s ? sg[qb] : s;
  return s;
}

// The entry words of one batch of rows [r, r + NB) of a lane's stream
// (rows at or past r1 read as padding).
template <int NB>
__device__ __forceinline__ void batch_ids(const uint2 *__restrict__ idx,
                                          int r, int r1, int lane,
                                          uint2 (&id)[NB]) {
#pragma unroll
  for (int u = 0; u < NB; ++u)
    id[u] = r + u < r1 ? idx[(size_t)(r + u) * kWave + lane]
                       : make_uint2(0u, 0u);
}

// The rest of a batch whose entry words id are loaded: na, nb, the numbers
// of the entry's two bins (zero exactly for inactive bins); on[u]: entry u
// is a pair of two active bins; its operands are loaded only then (and the
// Courant number only if with_c).
template <int NB, typename Real, typename Real2, typename RealC>
__device__ __forceinline__ void batch_fetch(
    const Real2 *__restrict__ ke, const Real2 *__restrict__ xe,
    const RealC *__restrict__ ce, bool with_c, int r, int lane,
    const Real *num, const uint2 (&id)[NB], bool (&on)[NB], Real (&na)[NB],
    Real (&nb)[NB], Real2 (&kb)[NB], Real2 (&xb)[NB], RealC (&cb)[NB]) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int qa = (int)(id[u].x & 0xffffu), qb = (int)(id[u].x >> 16);
    na[u] = num[qa];
    nb[u] = num[qb];
    on[u] = ((id[u].y >> 16) & kWValid) != 0 && na[u] != (Real)0 &&
            nb[u] != (Real)0;
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    if (!on[u]) continue;
    const size_t pos = (size_t)(r + u) * kWave + lane;
    kb[u] = ke[pos];
    xb[u] = xe[pos];
    if (with_c) cb[u] = ce[pos];
  }
}

// Byte offset of the shared-bin partial sums in a wave's LDS (after the
// per-bin arrays, 8-byte aligned), and the wave's LDS size.
template <bool F32>
__host__ __device__ constexpr size_t wave_part_offset(int SB) {
  return F32 ? ((((size_t)SB * 12 + 7) & ~(size_t)7) + (size_t)SB * 36 + 7) &
                   ~(size_t)7
             : (size_t)SB * 64;
}
// [3 accumulators][2 slots][64 lanes]: gain, outgoing flux and dneg of the
// gain pass; the loss pass reuses the first accumulator's slots, since its
// writes come after the barrier that ends the gain pass's last fix-up (a
// block without shared bins writes and reads no partial).
constexpr size_t kWavePartBytes = 3 * 2 * kWave * sizeof(double);

// Per-bin accumulators of a pass in LDS, FP64 in both modes.
struct PassLds {
  double *gain, *fout, *loss, *dneg;
  // a bin's entries of one species-pair block, added to its sum
  template <typename Acc>
  __device__ void merge(double *arr, int q, const Acc &a) const {
    arr[q] += a.val();
  }
  __device__ double read(const double *arr, int q) const { return arr[q]; }
};

// One step of one point by one wave (S1-S6).  Returns 1 if the limiter ran;
// in FP32C mode it returns 2 and leaves the point untouched when the
// limiter is needed (the caller takes that step in FP64 mode).  PF: load
// the next batch's entry words while the current batch's operands are in
// flight (it costs registers: the builds with room for them use it).
// OWN: bins a lane owns at most (the grid's schedule fits it).
template <bool F32, bool PF, int OWN>
__device__ unsigned point_step(const DevModel &m, const short *own_in,
                               double *st, int qs, double w, int br,
                               double dt, unsigned char *lds,
                               unsigned long long &npairs) {
  // owned bins, opaque per step: keeps the compiler from holding per-bin
  // addresses in registers across steps
  int own[OWN];
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    own[o] = own_in[o];
    asm volatile("" : "+v"(own[o]));
  }
  typedef typename std::conditional<F32, AccF32, AccF64>::type Acc;
  typedef typename std::conditional<F32, float, double>::type Real;
  typedef typename std::conditional<F32, float2, double2>::type Real2;
  const int lane = threadIdx.x;
  const int B = m.B, S = m.S, SB = m.S * m.B;
  // LDS: masses, numbers and log-masses (3 SB Real, at offset 0 so that a
  // bin's address is its index scaled), then the FP64 pass sums (4 SB
  // doubles from the next 8-byte boundary), then the limiter factors (FP64
  // mode, SB doubles) or the exponents of the split mass logs (FP32 mode,
  // SB ints); wave_part_offset gives the total
  Real *mass = (Real *)lds;
  Real *nv = mass + SB;
  Real *lnm = nv + SB;
  PassLds P;
  P.gain = (double *)(lds + ((3 * SB * sizeof(Real) + 7) & ~(size_t)7));
  P.fout = P.gain + SB;
  P.loss = P.gain + 2 * SB;
  P.dneg = P.gain + 3 * SB;
  double *sg = P.gain + 4 * SB;
  int *lne = (int *)(P.gain + 4 * SB);
  // partial sums of shared bins: [3 accumulators][2 slots][64 lanes], from
  // the next 8-byte boundary after the per-bin arrays (kWavePartBytes)
  double *psum = (double *)(lds + wave_part_offset<F32>(SB));

  // S1/S2: owned bins, FP64 total, activity.  The numbers and bin masses
  // of all owned bins are fetched before any is used; the bin k of
  // q = species B + k comes from one multiply (bmagic).
  double no[OWN], xo[OWN];
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    const int q = own[o];
    const unsigned qq = q < 0 ? 0u : (unsigned)q;
    const unsigned k = qq - __umulhi(qq, m.bmagic) * (unsigned)B;
    no[o] = q < 0 ? 0.0 : st[(size_t)qq * qs];
    xo[o] = m.x[k];
  }
  double part = 0.0;
#pragma unroll
  for (int o = 0; o < OWN; ++o)
    if (own[o] >= 0) part += no[o] * xo[o];
  const double Mtot = wave_sum_f64(part);
  const double thr = m.theta * Mtot;
  const double inv = Mtot > 0.0 ? 1.0 / Mtot : 0.0;
  uint64_t pres = 0;  // species with an active bin owned by this lane
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    const double Mq = no[o] * xo[o];
    const bool act = Mq > 0.0 && Mq >= thr;
    if (act) pres |= 1ull << __umulhi((unsigned)q, m.bmagic);
    const double Mt = act ? Mq : 0.0;
    if constexpr (F32) {
      const float mq = (float)(Mt * inv);
      mass[q] = mq;
      nv[q] = (float)((act ? no[o] : 0.0) * inv);
      log2_split(mq, lne[q], lnm[q]);
    } else {
      mass[q] = Mt;
      nv[q] = act ? no[o] : 0.0;
      lnm[q] = log_f64(Mt);
    }
    // the pass sums of a bin with no entries stay zero (its owner writes
    // every other bin's sums in the passes)
    P.gain[q] = P.fout[q] = P.loss[q] = P.dneg[q] = 0.0;
  }
  __syncthreads();
  // species present at this point: pairs of absent species are skipped
  // block by block (wave-uniform)
  pres = wave_or64(pres);
  Real wr, tdt;
  if constexpr (F32) {
    wr = (float)w;
    tdt = (float)(dt * Mtot);
  } else {
    wr = w;
    tdt = dt;
  }
  const size_t nrows = (size_t)(m.wrows_g + m.wrows_l) * kWave;
  const Real2 *xe;
  const Real2 *ke;
  if constexpr (F32) {
    xe = m.we_x32;
    ke = m.we_k32 + (size_t)br * nrows;
  } else {
    xe = m.we_x64;
    ke = m.we_k64 + (size_t)br * nrows;
  }

  typedef typename std::conditional<F32, float2, double>::type RealC;
  const RealC *ce;
  if constexpr (F32)
    ce = m.we_c32;
  else
    ce = m.we_c64;

  // rows per batch (FP64 operands take twice the registers)
  constexpr int NB = F32 ? 4 : 2;

  bool lim = false;
  for (int pass = 0; pass < 2; ++pass) {
    // S3/S4 gains over this lane's gain stream, species pair by pair.  The
    // stream is walked NB rows at a time: the rows' entry words, then
    // the masses of their bins, then the operands of the active entries
    // are each fetched for the whole batch before any of them is used, so
    // a batch waits for about two memory latencies instead of two per row.
    for (int sa = 0, ab = 0; sa < S; ++sa)
      for (int sb = sa; sb < S; ++sb, ++ab) {
        if (!((pres >> sa) & (pres >> sb) & 1ull)) continue;
        const int r0 = m.wblk[ab * 4], r1 = r0 + m.wblk[ab * 4 + 1];
        Acc g, f, d;
        g.zero();
        f.zero();
        d.zero();
        int cur = -1;
        bool cur_shared = false, first_flush = true;
        // FP32C: the current target's mass and its next bin's split log
        float mq = 0.0f, lm1 = 0.0f;
        int le1 = 0;
        // a bin's sums go to LDS directly, or (shared bin) to this lane's
        // slot: 0 for the first bin of its segment, 1 for the last
        auto flush = [&]() {
          if (cur < 0) return;
          if (cur_shared) {
            const int sl = first_flush ? 0 : 1;
            psum[(0 * 2 + sl) * kWave + lane] = g.val();
            psum[(1 * 2 + sl) * kWave + lane] = f.val();
            psum[(2 * 2 + sl) * kWave + lane] = d.val();
          } else {
            // the three sums read before any is written back
            const double g0 = P.gain[cur], f0 = P.fout[cur];
            const double d0 = pass == 0 ? P.dneg[cur] : 0.0;
            P.gain[cur] = g0 + g.val();
            P.fout[cur] = f0 + f.val();
            if (pass == 0) P.dneg[cur] = d0 + d.val();
          }
          first_flush = false;
        };
        uint2 idn[NB];
        if constexpr (PF) batch_ids<NB>(m.we_idx, r0, r1, lane, idn);
        for (int r = r0; r < r1; r += NB) {
          uint2 id[NB];
          bool on[NB];
          Real na[NB], nb[NB];
          Real2 kb[NB], xb[NB];
          RealC cb[NB];
          if constexpr (PF) {
#pragma unroll
            for (int u = 0; u < NB; ++u) id[u] = idn[u];
          } else {
            batch_ids<NB>(m.we_idx, r, r1, lane, id);
          }
          batch_fetch<NB>(ke, xe, ce, true, r, lane, nv, id, on, na, nb, kb,
                          xb, cb);
          if constexpr (PF) batch_ids<NB>(m.we_idx, r + NB, r1, lane, idn);
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const unsigned fl = id[u].y >> 16;
            if (!(fl & kWValid)) continue;  // padding at the block's end
            const int qt = (int)(id[u].y & 0xffffu);
            if (qt != cur) {
              flush();
              cur = qt;
              cur_shared = (fl & kWShared) != 0;
              g.zero();
              f.zero();
              d.zero();
              if constexpr (F32) {
                // the flux flag is the target's (not its species' top bin),
                // so it holds for the whole run
                if (fl & kWFlux) {
                  mq = mass[qt];
                  le1 = lne[qt + 1];
                  lm1 = lnm[qt + 1];
                }
              }
            }
            if (!on[u]) continue;
            const int qa = (int)(id[u].x & 0xffffu), qb = (int)(id[u].x >> 16);
            Real A, Bm;
            entry_amounts(fma(kb[u].y, wr, kb[u].x), tdt, na[u], nb[u],
                          (fl & kWSelf) != 0, xb[u], A, Bm);
            Real F;
            if constexpr (F32)
              F = (fl & kWFlux) ? entry_flux_f32(mq, le1, lm1, cb[u], A + Bm)
                                : 0.0f;
            else
              F = entry_flux((fl & kWFlux) != 0, mass, lnm, qt, cb[u],
                             A + Bm);
            const bool ta = (fl & kWTA) != 0, tb = (fl & kWTB) != 0;
            if constexpr (!F32) {  // second pass: FP64 mode only
              if (pass == 1) {
                const double sc =
                    pair_scale((const double *)sg, qa, qb, ta, tb, A, Bm, F);
                A *= sc;
                Bm *= sc;
                F *= sc;
              }
            }
            if constexpr (F32) {
              // exact transfers: the same rounded amounts as the source side
              if (!ta) g.add(A);
              if (!tb) g.add(Bm);
              g.add(-F);
            } else {
              // the pair's combined contribution to its target in one
              // rounding (a target that is also a source keeps the other
              // source's mass)
              const double keep = ta ? Bm : (tb ? A : A + Bm);
              g.add(keep - F);
            }
            f.add(F);
            if (pass == 0) {
              if (ta || tb) {
                const Real keep = ta ? Bm : A;
                if (F > keep) d.add(F - keep);
              }
              ++npairs;
            }
          }
        }
        flush();
        // fix-up: each shared bin's partials summed in lane order
        const int fo = m.wfixb[ab * 4], fn = m.wfixb[ab * 4 + 1];
        if (fn > 0) {
          __syncthreads();
          for (int t = lane; t < fn; t += kWave) {
            const uint2 fx = m.wfix[fo + t];
            const int q = (int)(fx.x & 0xffffu), l0 = (int)(fx.x >> 16);
            const int l1 = (int)(fx.y & 0xffffu), s0 = (int)(fx.y >> 16);
            double sg0 = psum[(0 * 2 + s0) * kWave + l0];
            double sf0 = psum[(1 * 2 + s0) * kWave + l0];
            double sd0 = psum[(2 * 2 + s0) * kWave + l0];
            for (int l = l0 + 1; l <= l1; ++l) {
              sg0 += psum[(0 * 2) * kWave + l];
              sf0 += psum[(1 * 2) * kWave + l];
              sd0 += psum[(2 * 2) * kWave + l];
            }
            P.gain[q] += sg0;
            P.fout[q] += sf0;
            if (pass == 0) P.dneg[q] += sd0;
          }
          __syncthreads();
        }
      }
    // losses over this lane's loss stream: the same collided amounts, seen
    // from the source bins (the Courant numbers only matter in the second
    // pass, where the pair's scale needs its flux)
    for (int sa = 0, ab = 0; sa < S; ++sa)
      for (int sb = sa; sb < S; ++sb, ++ab) {
        if (!((pres >> sa) & (pres >> sb) & 1ull)) continue;
        const int r0 = m.wblk[ab * 4 + 2], r1 = r0 + m.wblk[ab * 4 + 3];
        Acc lo;
        lo.zero();
        int cur = -1;
        bool cur_shared = false, first_flush = true;
        auto flush = [&]() {
          if (cur < 0) return;
          if (cur_shared)
            psum[(0 * 2 + (first_flush ? 0 : 1)) * kWave + lane] = lo.val();
          else
            P.merge(P.loss, cur, lo);
          first_flush = false;
        };
        uint2 idn[NB];
        if constexpr (PF) batch_ids<NB>(m.we_idx, r0, r1, lane, idn);
        for (int r = r0; r < r1; r += NB) {
          uint2 id[NB];
          bool on[NB];
          Real na[NB], nb[NB];
          Real2 kb[NB], xb[NB];
          RealC cb[NB];
          if constexpr (PF) {
#pragma unroll
            for (int u = 0; u < NB; ++u) id[u] = idn[u];
          } else {
            batch_ids<NB>(m.we_idx, r, r1, lane, id);
          }
          batch_fetch<NB>(ke, xe, ce, pass == 1, r, lane, nv, id, on, na, nb,
                          kb, xb, cb);
          if constexpr (PF) batch_ids<NB>(m.we_idx, r + NB, r1, lane, idn);
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const unsigned fl = id[u].y >> 16;
            if (!(fl & kWValid)) continue;
            const int qa = (int)(id[u].x & 0xffffu), qb = (int)(id[u].x >> 16);
            const bool sideb = (fl & kWSideB) != 0;
            const int q = sideb ? qb : qa;
            if (q != cur) {
              flush();
              cur = q;
              cur_shared = (fl & kWShared) != 0;
              lo.zero();
            }
            if (!on[u]) continue;
            const bool self = (fl & kWSelf) != 0;
            Real A, Bm;
            entry_amounts(fma(kb[u].y, wr, kb[u].x), tdt, na[u], nb[u],
                          self, xb[u], A, Bm);
            // the second pass runs in FP64 mode only: an FP32C step that
            // needs the limiter leaves the point to FP64 mode
            if constexpr (!F32) {
              if (pass == 1) {
                // the pair's scale, as its target's owner computes it
                const bool ta = (fl & kWTA) != 0, tb = (fl & kWTB) != 0;
                const int qt = (int)(id[u].y & 0xffffu);
                double F = 0.0;
                if (ta || tb)
                  F = entry_flux((fl & kWFlux) != 0, mass, lnm, qt, cb[u],
                                 A + Bm);
                const double sc =
                    pair_scale((const double *)sg, qa, qb, ta, tb, A, Bm, F);
                A *= sc;
                Bm *= sc;
              }
            }
            if (self) {
              lo.add(A);
              lo.add(Bm);
            } else {
              lo.add(sideb ? Bm : A);
            }
          }
        }
        flush();
        const int fo = m.wfixb[ab * 4 + 2], fn = m.wfixb[ab * 4 + 3];
        if (fn > 0) {
          __syncthreads();
          for (int t = lane; t < fn; t += kWave) {
            const uint2 fx = m.wfix[fo + t];
            const int q = (int)(fx.x & 0xffffu), l0 = (int)(fx.x >> 16);
            const int l1 = (int)(fx.y & 0xffffu), s0 = (int)(fx.y >> 16);
            double sl = psum[(0 * 2 + s0) * kWave + l0];
            for (int l = l0 + 1; l <= l1; ++l) sl += psum[(0 * 2) * kWave + l];
            P.loss[q] += sl;
          }
          __syncthreads();
        }
      }
    // every pass sum and outgoing flux visible to all lanes
    __syncthreads();
    if (pass == 1) break;
    // S5: demand of each owned bin = its negative merged nets; sigma where
    // the demand exceeds the mass.  FP32C also leaves the step to FP64 mode
    // when a bin would lose more than kDrainFp32 of its mass: the remainder
    // M - D of a draining bin is then small against D, and FP32 amounts
    // (inputs and arithmetic good to ~1e-7 of D) would carry a relative
    // error of ~1e-7 D / (M - D) into it, step after step.
    bool over = false;
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
      const int q = own[o];
      if (q < 0) continue;
      const double Mq = (double)mass[q];
      const double D = P.read(P.loss, q) + P.read(P.dneg, q);
      const bool od = F32 ? (D > kDrainFp32 * Mq) : (D > Mq);
      over = over || od;
      if constexpr (!F32) sg[q] = od ? Mq / D : 1.0;
    }
    lim = __any(over);
    if (!lim) break;
    if constexpr (F32) {
      __syncthreads();  // LDS is rewritten by the next step
      return 2u;
    }
    // the second pass sums start from zero again
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
      const int q = own[o];
      if (q < 0) continue;
      P.gain[q] = P.fout[q] = P.loss[q] = 0.0;
    }
    __syncthreads();  // sigma visible before the second pass
  }

  // S6: FP64 update of the owned bins
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    const int q = own[o];
    if (q < 0) continue;
    const int k = q - (int)__umulhi((unsigned)q, m.bmagic) * B;
    double gq = P.gain[q];
    if (k != 0) gq += P.fout[q - 1];
    double net = gq - P.read(P.loss, q);
    if constexpr (F32) net *= Mtot;
    const double xq = m.x[k];
    double Mn = st[(size_t)q * qs] * xq + net;
    Mn = Mn < 0.0 ? 0.0 : Mn;
    st[(size_t)q * qs] = Mn / xq;
  }
  __syncthreads();  // LDS is rewritten by the next step
  return lim ? 1u : 0u;
}

// The steps of one slot: a launch's steps (FP32C: until a step needs the
// limiter or drains a bin, then the slot is marked pending with the steps
// of the call left), or the pending steps in FP64 mode.
template <bool F32, bool PF, int OWN>
__device__ __forceinline__ void slot_steps(const WaveArgs &a,
                                           const WaveGrid &G,
                                           const short *own, int slot,
                                           int pend, unsigned char *lds,
                                           unsigned long long &npairs,
                                           unsigned long long &nlim,
                                           unsigned long long &nfp64) {
  const DevModel &m = G.m;
  const int SB = m.S * m.B;
  // bucket of the slot: its pressure bracket, or (points of the
  // multi-species lane kernels) bracket x species set
  const int nmask = G.tiled ? m.nmask : 1;
  int bk = 0;
  for (int b = 1; b < m.nbr * nmask; ++b)
    if (slot >= G.meta->bucket_base[b]) bk = b;
  const int br = bk / nmask;
  const double w = G.wgt[slot];
  // a point's bins: contiguous, or (tiled) 64 slots apart
  double *st = G.tiled ? G.state + state_index(0, slot, SB)
                       : G.state + (size_t)slot * SB;
  const int qs = G.tiled ? kWave : 1;
  const int n = a.pending_only ? pend : a.nsteps;
  for (int step = 0; step < n; ++step) {
    const unsigned r =
        point_step<F32, PF, OWN>(m, own, st, qs, w, br, a.dt, lds, npairs);
    if (F32 && r == 2u) {
      if (threadIdx.x == 0) G.pending[slot] = a.steps_left - step;
      break;
    }
    nlim += r;
  }
  if (a.pending_only) {
    nfp64 += (unsigned long long)pend;
    if (threadIdx.x == 0) G.pending[slot] = 0;
  }
}

// Builds that load the next batch's entry words ahead: those whose
// registers hold them without spilling into the pair loops.
constexpr bool wave_prefetch(bool f32, int w, int own) {
  return f32 ? (w == 3 || own <= kOwnSmall) : w == 2;
}

// Persistent waves over the compacted slots of every grid, handed out one
// at a time from a counter (counters[3], zero at the start of the call): a
// point's cost varies with its species and spectrum, and the FP64 steps of
// pending points are few and of very different lengths, so waves take work
// as they free up.  Every wave's loop ends on exactly one fetch past the
// last slot, so launch k of a call starts its numbering at k (slots +
// waves).  FP32C: a point whose step needs the limiter is marked pending
// (steps of the call left) and skipped from then on; pending_only: FP64
// steps for the marked points.
// Occupancy targets: FP32C mode fits 128 VGPRs, i.e. 4 waves per SIMD
// where the point's LDS allows it (four species: 3.2% faster than at 138
// VGPRs and 3 waves); FP64 mode at 168 VGPRs, 3 waves per SIMD, spills
// some registers and is still about 20% faster than at 238 VGPRs and 2
// waves (the entries' memory latency needs the waves).  Where the LDS of a
// point already holds a CU below 3 waves per SIMD, the spills buy nothing,
// and the FP64 build at 2 waves runs instead, with the entry words of the
// next batch loaded ahead (a few registers spilled outside the pair loops;
// 8% faster at 2 species x 132 bins, while at 3 waves the same prefetch
// spills into them and four species ran 7% slower); where it holds a CU to
// 12 waves or fewer (no SIMD can get a fourth), FP32C mode runs at 3 waves
// (0.9% faster at 2 species x 132 bins than at 4), where its registers
// leave room for the prefetch as well (145 VGPRs; 6% faster at 132 bins,
// 11% at 264).
template <bool F32, int W, int OWN>
__global__ void __launch_bounds__(kWave)
    __attribute__((amdgpu_waves_per_eu(W))) wave_step(WaveArgs a) {
  extern __shared__ unsigned char lds[];
  unsigned long long npairs = 0, nlim = 0, nfp64 = 0;
  long long total = 0;
  for (int g = 0; g < a.ngrids; ++g) total += a.g[g].meta->nslots;
  const unsigned long long base =
      (unsigned long long)a.launch_idx *
      (unsigned long long)(total + (long long)gridDim.x);
  int gown = -1;
  short own[OWN];
  for (;;) {
    unsigned long long t = 0;
    if (threadIdx.x == 0) t = atomicAdd(&a.counters[3], 1ull);
    // slot numbers of a launch stay below 2^31 (slots are int-indexed)
    int rem = uniform((int)(__shfl(t, 0) - base));
    int g = 0;
    while (g < a.ngrids && rem >= a.g[g].meta->nslots) {
      rem -= a.g[g].meta->nslots;
      ++g;
    }
    g = uniform(g);
    if (g >= a.ngrids) break;
    const WaveGrid &G = a.g[g];
    const int slot = uniform(rem);
    if (G.slot_point[slot] < 0) continue;  // padding
    const int pv = uniform(G.pending[slot]);
    if (a.pending_only ? pv <= 0 : pv != 0) continue;
    if (g != gown) {
#pragma unroll
      for (int o = 0; o < OWN; ++o)
        own[o] = G.m.own[threadIdx.x * kMaxOwn + o];
      gown = g;
    }
    slot_steps<F32, wave_prefetch(F32, W, OWN), OWN>(a, G, own, slot, pv, lds,
                                                     npairs, nlim, nfp64);
  }
  npairs = wave_sum_u64(npairs);
  if (threadIdx.x == 0) {
    if (npairs) atomicAdd(&a.counters[0], npairs);
    // pairs of the FP64 follow-up of FP32C points, counted apart as well
    if (npairs && a.pending_only) atomicAdd(&a.counters[4], npairs);
    if (nlim) atomicAdd(&a.counters[1], nlim);
    if (nfp64) atomicAdd(&a.counters[2], nfp64);
  }
}

// The build for the launch's occupancy target, by the bins a lane owns.
template <bool F32, int W>
void launch_own(const WaveArgs &a, int own, int blocks, size_t lds,
                hipStream_t st) {
  if (own <= kOwnSmall)
    hipLaunchKernelGGL((wave_step<F32, W, kOwnSmall>), dim3(blocks),
                       dim3(kWave), lds, st, a);
  else if (own <= kOwnMid)
    hipLaunchKernelGGL((wave_step<F32, W, kOwnMid>), dim3(blocks),
                       dim3(kWave), lds, st, a);
  else
    hipLaunchKernelGGL((wave_step<F32, W, kMaxOwn>), dim3(blocks),
                       dim3(kWave), lds, st, a);
}

}  // namespace

hipError_t launch_wave_step(const WaveArgs &a, int precision, int blocks,
                            hipStream_t st) {
  int sb = 0, own = 0;
  for (int g = 0; g < a.ngrids; ++g) {
    sb = a.g[g].m.S * a.g[g].m.B > sb ? a.g[g].m.S * a.g[g].m.B : sb;
    own = a.g[g].m.wown > own ? a.g[g].m.wown : own;
  }
  if (own < 1 || own > kMaxOwn) return hipErrorInvalidValue;
  // LDS per wave (see point_step): 3 Real per bin, padded to 8 bytes, 4
  // FP64 sums and a limiter factor (FP64) or an exponent (FP32C) per bin,
  // then the partial sums of shared bins
  const bool f64 = precision == 0 || a.pending_only;
  const size_t lds = (f64 ? wave_part_offset<false>(sb)
                          : wave_part_offset<true>(sb)) +
                     kWavePartBytes;
  // 3 waves per SIMD are 12 waves per CU, sharing its 160 KB of LDS; a
  // fourth wave on some SIMD needs room for 13
  constexpr size_t kLdsPerCu = 160 * 1024;
  if (f64 && lds * 12 <= kLdsPerCu)
    launch_own<false, 3>(a, own, blocks, lds, st);
  else if (f64)
    launch_own<false, 2>(a, own, blocks, lds, st);
  else if (lds * 13 <= kLdsPerCu)
    launch_own<true, 4>(a, own, blocks, lds, st);
  else
    launch_own<true, 3>(a, own, blocks, lds, st);
  return hipGetLastError();
}

}  // namespace fsbm
