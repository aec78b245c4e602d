// Host check of log_f64 (fp64_math.hpp): the same source the kernels
// compile, run on the CPU against the C library's log.  Prints the largest
// error in units in the last place over 10^7 seeded arguments (log-uniform
// over [1e-300, 1e10], and within 5e-4 of 1, where the result is small),
// then the special values.  Exit status 0.
#include <cmath>
#include <cstdio>
#include <random>

#include "../fp64_math.hpp"

static double ulps(double got, double ref) {
  if (got == ref) return 0.0;
  if (std::isnan(got) || std::isnan(ref) || std::isinf(got) ||
      std::isinf(ref))
    return 1e300;
  int e;
  std::frexp(ref, &e);
  return std::fabs(got - ref) / std::ldexp(1.0, e - 53);
}

int main() {
  std::mt19937_64 g(20240907);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  double worst = 0.0, at = 1.0;
  for (long i = 0; i < 10000000; ++i) {
    const double x =
        (i % 3 == 0) ? 1.0 + (U(g) - 0.5) * 1e-3 * std::pow(10.0, -6 * U(g))
                     : std::pow(10.0, -300.0 + 310.0 * U(g));
    const double d = ulps(fsbm::log_f64(x), std::log(x));
    if (d > worst) {
      worst = d;
      at = x;
    }
  }
  std::printf("max_ulp %.3f at %a\n", worst, at);
  const double sp[] = {0.0, INFINITY, -1.0, 4.9e-324, 2.2250738585072014e-308,
                       1.0, 2.0, 1e308};
  for (double v : sp)
    std::printf("special %a %a %a\n", v, fsbm::log_f64(v), std::log(v));
  return 0;
}
