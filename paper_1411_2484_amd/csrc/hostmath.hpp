// Host-side number theory for instance set-up: Montgomery arithmetic over
// 64-bit words, deterministic Rabin-Miller, inverses, discrete logarithms in
// the skip group and the SplitMix64 seeding stream.  None of this runs per
// draw; it prepares the per-instance constants the device kernels consume.
#pragma once

#include <cstdint>
#include <vector>

namespace phprng {

using u128 = unsigned __int128;

// Montgomery arithmetic modulo an odd n < 2^64 with R = 2^64.
struct Mont64 {
  uint64_t n = 0;
  uint64_t ninv = 0;  // n^{-1} mod 2^64
  uint64_t r1 = 0;    // R mod n
  uint64_t r2 = 0;    // R^2 mod n

  explicit Mont64(uint64_t modulus) : n(modulus) {
    // Newton iteration for the inverse of an odd number modulo 2^64.
    uint64_t x = n;  // correct to 3 bits
    for (int i = 0; i < 5; ++i) x *= 2 - n * x;
    ninv = x;
    // R mod n by doubling 1 sixty-four times, R^2 mod n by 64 more doublings.
    uint64_t v = 1 % n;
    for (int i = 0; i < 64; ++i) v = add(v, v);
    r1 = v;
    for (int i = 0; i < 64; ++i) v = add(v, v);
    r2 = v;
  }
  uint64_t add(uint64_t x, uint64_t y) const {  // x, y < n
    uint64_t s = x + y;
    bool carry = s < x;
    return (carry || s >= n) ? s - n : s;
  }
  uint64_t sub(uint64_t x, uint64_t y) const { return x >= y ? x - y : x + (n - y); }
  // x * y * R^{-1} mod n for x, y < n.
  uint64_t mul(uint64_t x, uint64_t y) const {
    u128 t = (u128)x * y;
    uint64_t lo = (uint64_t)t, hi = (uint64_t)(t >> 64);
    uint64_t q = lo * ninv;
    uint64_t qh = (uint64_t)(((u128)q * n) >> 64);
    return hi >= qh ? hi - qh : hi + (n - qh);
  }
  uint64_t to(uint64_t x) const { return mul(x % n, r2); }
  uint64_t from(uint64_t x) const { return mul(x, 1); }
  uint64_t pow_m(uint64_t base_m, uint64_t e) const {  // Montgomery in, Montgomery out
    uint64_t r = r1;
    while (e) {
      if (e & 1) r = mul(r, base_m);
      base_m = mul(base_m, base_m);
      e >>= 1;
    }
    return r;
  }
  uint64_t mulmod(uint64_t x, uint64_t y) const { return from(mul(to(x), to(y))); }
  uint64_t powmod(uint64_t b, uint64_t e) const { return from(pow_m(to(b), e)); }
  // Reduce a 128-bit value: v mod n = REDC(REDC(v) * R^2) for v < n * 2^64.
  uint64_t reduce128(u128 v) const;
};

uint64_t gcd64(uint64_t a, uint64_t b);
// Inverse of a modulo m (m >= 2); returns 0 when gcd(a, m) != 1.
uint64_t inverse_mod(uint64_t a, uint64_t m);
bool is_prime64(uint64_t n);

// SplitMix64 output function (Steele, Lea and Flood, 2014).
inline uint64_t splitmix64(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Skip group data for one width: p, a, the factorisation of p - 1 and the
// inverse a^{-1} mod p.  Discrete logarithm t with a^t = s mod p by
// Pohlig-Hellman over the prime-power factors of p - 1 (all small).
struct SkipGroup {
  uint64_t p = 0, a = 0, ainv = 0;
  std::vector<uint64_t> primes;  // prime factors of p - 1
  std::vector<int> exps;         // their multiplicities
  SkipGroup(uint64_t p_, uint64_t a_);
  uint64_t mulmod(uint64_t x, uint64_t y) const;
  uint64_t powmod(uint64_t b, uint64_t e) const;
  // t in [0, p-2] with a^t = s (mod p), s in [1, p-1].
  uint64_t dlog(uint64_t s) const;
};

}  // namespace phprng
