// Host check of the FP64 power function of csrc/fp64math.hpp against the host
// C library: relative error of x^e over x in [1e-6, 1e6] (log-uniform) and
// e in [-2, 2], and of ln and exp on their own.  Exit status 0 when the largest
// relative error is below 1e-14.
#include <cmath>
#include <cstdio>
#include <random>

#include "fp64math.hpp"

int main() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> ux(-6.0, 6.0), ue(-2.0, 2.0), ut(-30.0, 30.0);
  double e_pow = 0.0, e_ln = 0.0, e_exp = 0.0;
  for (int i = 0; i < 200000; ++i) {
    const double x = std::pow(10.0, ux(rng)), e = ue(rng), t = ut(rng);
    const double p = lbm::pow_pos(x, e), pr = std::pow(x, e);
    e_pow = std::fmax(e_pow, std::fabs(p - pr) / pr);
    const double l = lbm::ln_pos(x), lr = std::log(x);
    e_ln = std::fmax(e_ln, std::fabs(l - lr) / std::fmax(std::fabs(lr), 1.0));
    const double q = lbm::exp_of(t), qr = std::exp(t);
    e_exp = std::fmax(e_exp, std::fabs(q - qr) / qr);
  }
  // the Carreau-Yasuda use: (1 + (lambda g)^2)^((n - 1)/2) near 1
  for (int i = 0; i < 100000; ++i) {
    const double la = std::pow(10.0, -12.0 + 13.0 * (i / 100000.0));
    const double p = lbm::pow_pos(1.0 + la, -0.32), pr = std::pow(1.0 + la, -0.32);
    e_pow = std::fmax(e_pow, std::fabs(p - pr) / pr);
  }
  std::printf("fp64math: max relative error pow %.3e, ln %.3e, exp %.3e\n", e_pow, e_ln, e_exp);
  return (e_pow < 1e-14 && e_ln < 1e-14 && e_exp < 1e-14) ? 0 : 1;
}
