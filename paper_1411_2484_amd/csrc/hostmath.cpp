// Host-side number theory (see hostmath.hpp).
#include "hostmath.hpp"

namespace phprng {

uint64_t Mont64::reduce128(u128 v) const {
  // REDC(v) = v R^{-1} mod n needs v < n R; then multiply by R^2.
  uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  uint64_t q = lo * ninv;
  uint64_t qh = (uint64_t)(((u128)q * n) >> 64);
  uint64_t r = hi >= qh ? hi - qh : hi + (n - qh);
  return mul(r, r2);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

uint64_t inverse_mod(uint64_t a, uint64_t m) {
  if (m < 2) return 0;
  // Iterative extended Euclid on (m, a mod m), coefficients kept mod m.
  uint64_t old_r = m, r = a % m;
  uint64_t old_s = 0, s = 1;  // old_s * a == old_r (mod m), s * a == r (mod m)
  while (r != 0) {
    uint64_t qt = old_r / r;
    uint64_t nr = old_r - qt * r;
    old_r = r;
    r = nr;
    // ns = old_s - qt * s  (mod m)
    uint64_t prod = (uint64_t)(((u128)qt * s) % m);
    uint64_t ns = old_s >= prod ? old_s - prod : old_s + (m - prod);
    old_s = s;
    s = ns;
  }
  if (old_r != 1) return 0;
  return old_s % m;
}

static const uint64_t kSmallPrimes[] = {2,  3,  5,  7,  11, 13, 17, 19, 23, 29, 31, 37, 41,
                                        43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

bool is_prime64(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t q : kSmallPrimes) {
    if (n == q) return true;
    if (n % q == 0) return false;
  }
  Mont64 M(n);
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++r;
  }
  const uint64_t one = M.r1, minus_one = M.sub(0, M.r1);
  const int nb = n < (1ull << 32) ? 5 : 12;
  for (int i = 0; i < nb; ++i) {
    uint64_t x = M.pow_m(M.to(kSmallPrimes[i]), d);
    if (x == one || x == minus_one) continue;
    bool witness = true;
    for (int j = 1; j < r; ++j) {
      x = M.mul(x, x);
      if (x == minus_one) {
        witness = false;
        break;
      }
    }
    if (witness) return false;
  }
  return true;
}

SkipGroup::SkipGroup(uint64_t p_, uint64_t a_) : p(p_), a(a_) {
  uint64_t m = p - 1;
  for (uint64_t q = 2; q * q <= m; ++q) {
    if (m % q == 0) {
      int e = 0;
      while (m % q == 0) {
        m /= q;
        ++e;
      }
      primes.push_back(q);
      exps.push_back(e);
    }
  }
  if (m > 1) {
    primes.push_back(m);
    exps.push_back(1);
  }
  ainv = inverse_mod(a, p);
}

uint64_t SkipGroup::mulmod(uint64_t x, uint64_t y) const { return (uint64_t)(((u128)x * y) % p); }

uint64_t SkipGroup::powmod(uint64_t b, uint64_t e) const {
  uint64_t r = 1;
  b %= p;
  while (e) {
    if (e & 1) r = mulmod(r, b);
    b = mulmod(b, b);
    e >>= 1;
  }
  return r;
}

uint64_t SkipGroup::dlog(uint64_t s) const {
  const uint64_t order = p - 1;
  // For each q^k || p-1: x mod q^k digit by digit (each digit by search over
  // the q-th roots of unity), then combine by the Chinese remainder theorem.
  u128 x_total = 0, mod_total = 1;
  for (size_t f = 0; f < primes.size(); ++f) {
    uint64_t q = primes[f];
    int k = exps[f];
    uint64_t qk = 1;
    for (int i = 0; i < k; ++i) qk *= q;
    uint64_t g = powmod(a, order / q);  // generator of the order-q subgroup
    // table of g^j, j < q (q is at most a few thousand)
    std::vector<uint64_t> gj(q);
    gj[0] = 1;
    for (uint64_t j = 1; j < q; ++j) gj[j] = mulmod(gj[j - 1], g);
    uint64_t x = 0, qpow = 1;  // x mod q^i so far
    for (int i = 0; i < k; ++i) {
      // h = (s * a^{-x})^{order / q^{i+1}}
      uint64_t h = mulmod(s, powmod(ainv, x));
      uint64_t ex = order / (qpow * q);
      h = powmod(h, ex);
      uint64_t d = 0;
      while (d < q && gj[d] != h) ++d;
      if (d == q) return ~0ull;  // s not in the group (cannot happen for 1 <= s < p)
      x += d * qpow;
      qpow *= q;
    }
    // CRT: find X = x_total (mod mod_total), X = x (mod qk)
    uint64_t mt = (uint64_t)(mod_total % qk);
    uint64_t inv = inverse_mod(mt, qk);
    uint64_t xt = (uint64_t)(x_total % qk);
    uint64_t diff = x >= xt ? x - xt : x + (qk - xt);
    uint64_t tcoef = (uint64_t)(((u128)diff * inv) % qk);
    x_total += mod_total * tcoef;
    mod_total *= qk;
  }
  return (uint64_t)(x_total % order);
}

}  // namespace phprng
