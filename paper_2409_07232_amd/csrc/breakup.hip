// breakup.hip -- spontaneous breakup of the drop spectrum (the first
// species): a drop of bin l breaks at the rate P_l into Q[l][k] fragments
// in each smaller bin k (the linear breakup equation of Srivastava 1971,
// with a breakup probability per unit time of the kind Komabayasi, Gonda
// and Isono 1964 fitted).  Over a step the share b_l = 1 - exp(-P_l dt) of
// bin l breaks, its fragments not breaking again within the step:
//   N'_k = (N_k - b_k N_k) + sum_{l>k} (b_l N_l) Q[l][k],  ascending l.
// The paper lists breakup among the process terms of the bin equation
// (Sec. III, eq. (1)).
//
// Mapping (gfx950): the points holding drops are compacted (the shared
// liquid compaction); at 33 and 66 bins one point per lane, its B bins in
// VGPRs for all steps of the call; b and the lower triangle of Q are wave-uniform and read
// through the scalar cache; every register index is static after
// unrolling, so the step is B^2 FP64 multiply and add pairs with no memory
// traffic.  At 66 bins the broken numbers b_l N_l are recomputed where they
// are used (the same product, so the same value) instead of held, which
// keeps the kernel within the register file.  Operations in the
// definition's order, products and sums not fused: the result is the
// definition's bit for bit.
#include "device_common.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

constexpr int kBrkThreads = 64;

// Q is held transposed on the device (QT[k][l] = Q[l][k]), so the
// fragments a bin k receives are one contiguous run of scalar loads; the
// table pointers are made opaque per bin so that the compiler loads each
// run where it is used instead of holding the whole table in SGPRs.
template <int B, bool HOLD>
__global__ void __launch_bounds__(kBrkThreads) brk_steps(BrkArgs a) {
  const int count = *a.count;
  const int slot = blockIdx.x * kBrkThreads + threadIdx.x;
  if (slot >= count) return;
  const int64_t pt = a.idx[slot];
  double *row = a.N + pt * a.SB;
  double n[B];
#pragma unroll
  for (int k = 0; k < B; ++k) n[k] = row[k];
  for (int st = 0; st < a.nsteps; ++st) {
    if (HOLD) {
      double L[B];
      const double *bq = a.b;
      asm volatile("" : "+s"(bq));
#pragma unroll
      for (int l = 0; l < B; ++l) L[l] = ldc(bq + l) * n[l];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const double *qk = a.QT + k * B;
        asm volatile("" : "+s"(qk));
        double v = n[k] - L[k];
#pragma unroll
        for (int l = k + 1; l < B; ++l) v += L[l] * ldc(qk + l);
        n[k] = v;
      }
    } else {
      // n[l] for l > k still holds the step's start value when bin k is
      // formed, so b_l n_l is the same product as the held form's
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const double *qk = a.QT + k * B;
        const double *bq = a.b;
        asm volatile("" : "+s"(qk));
        asm volatile("" : "+s"(bq));
        double v = n[k] - ldc(bq + k) * n[k];
#pragma unroll
        for (int l = k + 1; l < B; ++l)
          v += (ldc(bq + l) * n[l]) * ldc(qk + l);
        n[k] = v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < B; ++k) row[k] = n[k];
}

// Grids beyond the lane kernel (67 to kMaxBins bins): one listed point
// per wave at a time (a grid of waves strides over the list), its bins in
// LDS.  Lane r of the wave forms bins k = r, r + 64, ... (R of them, held
// in registers); the rows l of the fragment table are walked in ascending
// order by all lanes together, so the wave reads row l's entries Q[l][k]
// for consecutive k in one access and each bin still sums its fragments in
// ascending l, the definition's order.
template <int R>
__global__ void __launch_bounds__(kBrkThreads) brk_wave(BrkArgs a) {
  extern __shared__ double lds[];
  const int B = a.B, lane = threadIdx.x;
  double *n = lds, *L = lds + B;
  const int count = *a.count;
  for (int slot = blockIdx.x; slot < count; slot += gridDim.x) {
    const int64_t pt = a.idx[slot];
    double *row = a.N + pt * a.SB;
    for (int k = lane; k < B; k += kBrkThreads) n[k] = row[k];
    __syncthreads();
    for (int st = 0; st < a.nsteps; ++st) {
      for (int l = lane; l < B; l += kBrkThreads) L[l] = a.b[l] * n[l];
      __syncthreads();
      double v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = lane + r * kBrkThreads;
        v[r] = k < B ? n[k] - L[k] : 0.0;
      }
      for (int l = 1; l < B; ++l) {
        const double Ll = L[l];
        const double *Ql = a.Q + (size_t)l * B;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int k = lane + r * kBrkThreads;
          if (k < l) v[r] += Ll * Ql[k];
        }
      }
      __syncthreads();  // every lane has read L and n before n changes
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = lane + r * kBrkThreads;
        if (k < B) n[k] = v[r];
      }
      __syncthreads();
    }
    for (int k = lane; k < B; k += kBrkThreads) row[k] = n[k];
    __syncthreads();
  }
}

template <int R>
hipError_t launch_wave_r(const BrkArgs &a, hipStream_t st) {
  const int64_t want = a.npoints < 2048 ? a.npoints : 2048;
  hipLaunchKernelGGL((brk_wave<R>), dim3((unsigned)want), dim3(kBrkThreads),
                     sizeof(double) * 2 * a.B, st, a);
  return hipGetLastError();
}

hipError_t launch_wave(const BrkArgs &a, hipStream_t st) {
  switch ((a.B + kBrkThreads - 1) / kBrkThreads) {
    case 2: return launch_wave_r<2>(a, st);
    case 3: return launch_wave_r<3>(a, st);
    case 4: return launch_wave_r<4>(a, st);
    case 5: return launch_wave_r<5>(a, st);
    case 6: return launch_wave_r<6>(a, st);
    case 7: return launch_wave_r<7>(a, st);
    case 8: return launch_wave_r<8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <int B, bool HOLD>
hipError_t launch_b(const BrkArgs &a, unsigned blocks, hipStream_t st) {
  hipLaunchKernelGGL((brk_steps<B, HOLD>), dim3(blocks), dim3(kBrkThreads),
                     0, st, a);
  return hipGetLastError();
}

}  // namespace

bool brk_supported(int B) {
  return B == 33 || B == 66 || (B > 66 && B <= kMaxBins);
}

hipError_t launch_breakup(const BrkArgs &a, hipStream_t st) {
  if (!brk_supported(a.B) || a.npoints > 0x7fffffffLL)
    return hipErrorInvalidValue;
  if (a.npoints == 0 || a.nsteps == 0) return hipSuccess;
  // points with drops in a bin that breaks (bins 1..B-1)
  hipError_t e = launch_liquid_compact(a.N, a.npoints, a.SB, a.B, 1, nullptr,
                                       nullptr, 0.0, a.idx, a.count, st);
  if (e != hipSuccess) return e;
  if (a.B > 66) return launch_wave(a, st);
  const unsigned blocks =
      (unsigned)((a.npoints + kBrkThreads - 1) / kBrkThreads);
  return a.B == 33 ? launch_b<33, true>(a, blocks, st)
                   : launch_b<66, false>(a, blocks, st);
}

}  // namespace fsbm
