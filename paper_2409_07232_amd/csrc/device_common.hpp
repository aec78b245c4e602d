// device_common.hpp -- small device helpers shared by the gfx950 kernels of
// the collision step: register-resident bin arrays with wave-uniform dynamic
// indexing, wave reductions, the split log2 and the flux fraction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fp64_math.hpp"
#include "fsbm_internal.hpp"

namespace fsbm {

// ---------------------------------------------------------------- arrays
// Per-lane bin arrays kept in VGPRs.  Vector chunks of at most 32 registers
// let the backend index them with a wave-uniform dynamic index
// (s_set_gpr_idx) instead of spilling to scratch; static indices after loop
// unrolling resolve to plain registers.
template <int N>
struct VecD {
  typedef double type __attribute__((ext_vector_type(N)));
};

template <int B>
struct BinsD {
  static_assert(B >= 2 && B <= 48, "BinsD holds 2..48 bins");
  static constexpr int N0 = B < 16 ? B : 16;
  static constexpr int N1 = B > 16 ? (B - 16 < 16 ? B - 16 : 16) : 1;
  static constexpr int N2 = B > 32 ? B - 32 : 1;
  typename VecD<N0>::type c0;
  typename VecD<N1>::type c1;
  typename VecD<N2>::type c2;
  __device__ __forceinline__ double get(int k) const {
    return (k < 16) ? c0[k] : ((k < 32) ? c1[k - 16] : c2[k - 32]);
  }
  __device__ __forceinline__ void set(int k, double v) {
    if (k < 16)
      c0[k] = v;
    else if (k < 32)
      c1[k - 16] = v;
    else
      c2[k - 32] = v;
  }
};

// ------------------------------------------------------- constant loads
// Read-only model tables are read through the constant address space, so
// wave-uniform addresses become scalar loads (s_load, scalar data cache).
template <typename T>
__device__ __forceinline__ T ldc(const T *p) {
  return *(const __attribute__((address_space(4))) T *)p;
}

// ----------------------------------------------------------- wave helpers
__device__ __forceinline__ int uniform(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    lo |= __shfl_xor(lo, o);
    hi |= __shfl_xor(hi, o);
  }
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(
    unsigned long long v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// log2 of x >= 0 split into an exact integer exponent e and the log2 of the
// mantissa in [1/2, 1) (f in [-1, 0)): a difference of two such logs is
// exact in its integer part, so it keeps ~1e-7 absolute accuracy where
// |log2 x| is large (a plain FP32 log2 of 1e-9 is only good to ~2e-6).
// The hardware log2 rounds toward -infinity, so a plain difference of two
// logs of different size carries a one-sided error of up to half an ulp
// of the larger (4e-6 near log2 = -100); split, it is below 3e-8.
__device__ __forceinline__ void log2_split(float x, int &e, float &f) {
  e = __builtin_amdgcn_frexp_expf(x);
  f = __builtin_amdgcn_logf(__builtin_amdgcn_frexp_mantf(x));
}

// ------------------------------------------------------- flux fraction
// f(c, x1) = integral over [1/2 - c, 1/2] of exp(x1 t) dt, clamped to
// [0, 1]: the fraction of the merged mass that an exponential sub-bin
// profile with log-slope x1 places above x_{k+1} - c (x_{k+1} - x_k).
// FP64 form: exp((1/2 - c) x1) expm1(c x1) / x1, with its x1 -> 0 limit c.
__device__ __forceinline__ double flux_fraction_f64(double c, double x1) {
  double f;
  if (c == 0.0) {
    f = 0.0;
  } else if (x1 == 0.0) {
    f = c;
  } else if (x1 > 700.0) {
    f = 1.0;  // f increases with x1 >= 0 and exceeds 1 here for c > 1e-150
  } else {
    f = exp((0.5 - c) * x1) * expm1(c * x1) / x1;
  }
  return fmin(fmax(f, 0.0), 1.0);
}

// FP32 form on the half base-2 log-slope h = x1 / (2 ln 2):
//   f = c 2^h g(y),  y = c x1 = ys h with ys = 2 c ln 2,  g(y) = (1 - e^-y) / y,
// with g from its Taylor series for |y| < 1/4 (truncation error below
// 5e-8) and from the hardware exp2 otherwise, where e^-y = 2^-(2 c h) and
// 2 c h = c h + c h exactly.  Carrying the half slope saves the multiply
// by 1/2 in front of the exp2.
// Errors here must be unbiased, not only small: the tail of a spectrum is
// built over many steps from fluxes of this form, so a one-sided error of
// 1e-7 in f adds up (measured: up to 2e-4 in bins holding 1e-9 of a
// point's mass).  The hardware reciprocal of a negative y rounds toward
// zero; one Newton step leaves a round-to-nearest error instead.
__device__ __forceinline__ float flux_fraction_half_f32(float c, float ys,
                                                        float h) {
  const float y = ys * h;
  const float e = __builtin_amdgcn_exp2f(h);
  float g;
  if (__builtin_fabsf(y) < 0.25f) {
    g = 1.0f + y * (-0.5f + y * (1.0f / 6.0f + y * (-1.0f / 24.0f +
                                                    y * (1.0f / 120.0f -
                                                         y * (1.0f / 720.0f)))));
  } else {
    float r = __builtin_amdgcn_rcpf(y);
    r = __builtin_fmaf(r, __builtin_fmaf(-y, r, 1.0f), r);
    const float u = c * h;
    g = (1.0f - __builtin_amdgcn_exp2f(-(u + u))) * r;
  }
  return __builtin_fminf(c * e * g, 1.0f);
}

// Half-slope bounds (base 2): the empty-neighbour floor x1 = kX1Floor, and
// a ceiling at x1 = 173 where f(c, x1) >= 1 already holds for every
// c >= 3e-38 (so the clamp of f decides) while 2^h stays finite.
constexpr float kHalfLamFloor = (float)(0.5 * kX1Floor / 0.69314718055994530942);
constexpr float kHalfLamCeil = (float)(0.5 * 173.0 / 0.69314718055994530942);

}  // namespace fsbm
