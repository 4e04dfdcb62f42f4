// x^e in FP64 for x > 0, for the Carreau-Yasuda law in the FP64 arithmetic of
// the adjoint's passes.  Classical range reductions (see e.g. J.-M. Muller,
// "Elementary Functions: Algorithms and Implementation"):
//   ln x  = k ln 2 + ln m,  x = m 2^k with m in [1/sqrt 2, sqrt 2),
//   ln m  = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1)/(m + 1),
//           |s| <= 0.1716, eleven terms (truncation below 1e-18);
//   2^y   = 2^j e^(f ln 2),  j = nearest integer to y, |f| <= 1/2, Taylor
//           polynomial of degree 13 of e^t for |t| <= 0.347 (truncation
//           below 1e-17), then a power-of-two scaling.
// About 35 FP64 operations and few registers; relative error a few units in
// the last place (checked against the host's pow by tests/sanitize).
#pragma once
#include <cmath>

namespace lbm {

__host__ __device__ inline double ln_pos(double x) {
  int k;
  double m = std::frexp(x, &k);  // x = m 2^k, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    k -= 1;
  }
  // s = (m - 1) / (m + 1): FP32 reciprocal refined by two Newton steps
  const double den = m + 1.0;
  double r = (double)(1.0f / (float)den);
  r = r * (2.0 - den * r);
  r = r * (2.0 - den * r);
  const double s = (m - 1.0) * r;
  const double z = s * s;
  // sum_{j=0}^{10} z^j / (2j + 1), by Horner
  double p = 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0;
  return (double)k * 0.69314718055994530942 + 2.0 * s * p;
}

__host__ __device__ inline double exp_of(double t) {
  // t = (j + f) ln 2
  const double y = t * 1.44269504088896340736;  // t / ln 2
  const double j = std::rint(y);
  const double r = (y - j) * 0.69314718055994530942;
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  return std::ldexp(p, (int)j);
}

// x^e for x > 0.
__host__ __device__ inline double pow_pos(double x, double e) { return exp_of(e * ln_pos(x)); }

}  // namespace lbm
