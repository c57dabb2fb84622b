// Host-side statistics shared by the battery and the pattern analysis: the
// regularised incomplete gamma function behind chi-square P-values.
#pragma once

#include <cmath>

namespace phprng {

// Regularised incomplete gamma: P(a, x) by its power series below x = a + 1,
// Q(a, x) by the Legendre continued fraction (modified Lentz evaluation)
// above.  The common factor x^a e^-x / Gamma(a+1) is formed as
// -a (t - log1p t) - log sqrt(2 pi a) - (Stirling remainder), t = x/a - 1,
// which keeps its accuracy for the 10^6 degrees of freedom of the large tests.
inline double log_prefactor(double a, double x) {
  if (a < 10.0) return a * std::log(x) - x - std::lgamma(a + 1.0);
  const double t = (x - a) / a;
  const double a2 = a * a;
  const double rem = 1.0 / (12.0 * a) - 1.0 / (360.0 * a * a2) + 1.0 / (1260.0 * a * a2 * a2) -
                     1.0 / (1680.0 * a * a2 * a2 * a2);
  const double two_pi = 6.283185307179586;
  return -a * (t - std::log1p(t)) - 0.5 * std::log(two_pi * a) - rem;
}

inline void gamma_pq(double a, double x, double *P, double *Q) {
  if (x <= 0.0) {
    *P = 0.0;
    *Q = 1.0;
    return;
  }
  const double lp = log_prefactor(a, x);
  if (x < a + 1.0) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 1000000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (term < sum * 1e-17) break;
    }
    *P = std::exp(lp) * sum;
    *Q = 1.0 - *P;
  } else {
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 1000000; ++i) {
      const double an = -i * (i - a);
      b += 2.0;
      d = an * d + b;
      if (std::fabs(d) < tiny) d = tiny;
      c = b + an / c;
      if (std::fabs(c) < tiny) c = tiny;
      d = 1.0 / d;
      const double del = d * c;
      h *= del;
      if (std::fabs(del - 1.0) < 1e-16) break;
    }
    *Q = std::exp(lp + std::log(a)) * h;  // x^a e^-x / Gamma(a)
    *P = 1.0 - *Q;
  }
}

}  // namespace phprng
