// fp64_math.hpp -- FP64 natural logarithm for the flux slope of the FP64
// collision paths, written from the atanh series.  The device library's
// log takes 84 VALU instructions on gfx950 (98 with its constant moves);
// this one 43, at an error of at most two units in the last place
// (measured against the host's C library over 10^7 arguments across
// [1e-300, 1e10] and near 1).  Host and device compile the same code, so
// the host check runs the device arithmetic.  (Series forms of exp and
// expm1 came to 26 and 28 instructions against the library's 23 and 32, so
// the library's are kept.)
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fsbm {

// ln 2 as a 42-bit head (e * head is exact for |e| < 2^11) and its tail
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

// log x = e ln 2 + 2 atanh(s) with x = 2^e m, m in [sqrt(1/2), sqrt(2)) and
// s = (m - 1) / (m + 1), |s| <= 0.1716 (m - 1 is exact): the atanh series
// 2 s (1 + s^2/3 + ... + s^18/19); the first omitted term is below 2^-55 of
// the sum.  log 0 = -inf, log inf = inf, log of a negative number or NaN is
// NaN.
__host__ __device__ inline double log_f64(double x) {
#pragma clang fp contract(off)
  int e;
  double m = frexp(x, &e);
  if (m < kSqrtHalf) {
    m = m + m;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 19.0;
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double ss = s + s;
  const double r = fma(ss * z, p, ss);  // 2 s + 2 s z p
  const double ed = (double)e;
  const double v = fma(ed, kLn2Hi, fma(ed, kLn2Lo, r));
  if (x > 0.0 && x < INFINITY) return v;
  return x == 0.0 ? -INFINITY : (x == INFINITY ? x : NAN);
}

}  // namespace fsbm
