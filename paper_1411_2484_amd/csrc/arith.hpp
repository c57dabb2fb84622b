// Device arithmetic for gfx950: Montgomery products over 32-bit words (and
// 64-bit moduli from 32-bit limbs), Mersenne reductions for the skip
// generators, and the wave-level helpers the kernels use.
//
// A 32 x 32 -> 64 product (plus a 64-bit addend) is one v_mad_u64_u32; on
// gfx950 it issues at about 60% of the rate of a plain 32-bit add, so the
// 64-bit routines below are arranged to need few of them and few carries
// (the one carry the Montgomery reduction cannot avoid is the
// multiply-add's own carry-out).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "layout.hpp"

namespace phprng {

// Clears the calling thread's last HIP error before a launch whose error is
// read with hipGetLastError: a call that failed earlier in the process (an
// allocation refused somewhere else, say) would otherwise be reported as
// this launch's failure.
inline void clear_launch_error() { (void)hipGetLastError(); }

namespace dev {

// ---- skip generator mod 2^31 - 1 (eq. (5), width 32) ----------------------

// x y mod (2^31 - 1) for x, y in [1, 2^31 - 2]: fold the 62-bit product.
__device__ __forceinline__ uint32_t mulmod_p31(uint32_t x, uint32_t y) {
  uint64_t t = (uint64_t)x * y;
  uint32_t v = ((uint32_t)t & 0x7fffffffu) + (uint32_t)(t >> 31);
  uint32_t w = v - 0x7fffffffu;
  return min(v, w);  // v < 2p, v != p: subtract p once when v > p
}

__device__ __forceinline__ uint32_t powmod_p31(uint32_t b, uint64_t e) {
  uint32_t r = 1;
  while (e) {
    if (e & 1) r = mulmod_p31(r, b);
    b = mulmod_p31(b, b);
    e >>= 1;
  }
  return r;
}

// One in an SGPR that the compiler cannot fold to a constant.
__device__ __forceinline__ uint32_t opaque_one() {
  uint32_t one;
  asm volatile("s_mov_b32 %0, 1" : "=s"(one));
  return one;
}

// acc + x as a single v_mad_u64_u32 (x * one + acc, one == 1): the 32-bit
// addend needs no zero-extended register pair.
__device__ __forceinline__ uint64_t acc_u32(uint64_t acc, uint32_t x, uint32_t one) {
  return (uint64_t)x * one + acc;
}

// ---- 32-bit Montgomery arithmetic modulo n in [2^31, 2^32) ----------------

// x y 2^{-32} mod n for x, y < n; ninv = n^{-1} mod 2^32.  The low words of
// x y and q n cancel exactly, so the result is hi(x y) - hi(q n) (+ n).
// Six VALU instructions: v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32,
// v_sub_co_u32 (borrow), v_cndmask_b32, v_add_u32.
__device__ __forceinline__ uint32_t mont32(uint32_t x, uint32_t y, uint32_t n, uint32_t ninv) {
  uint64_t t = (uint64_t)x * y;
  uint32_t q = (uint32_t)t * ninv;
  uint32_t qh = __umulhi(q, n);
  uint32_t r;
  bool borrow = __builtin_usub_overflow((uint32_t)(t >> 32), qh, &r);
  return r + (borrow ? n : 0u);
}

// v 2^{-32} mod n for v < n 2^32.
__device__ __forceinline__ uint32_t redc32(uint64_t v, uint32_t n, uint32_t ninv) {
  uint32_t q = (uint32_t)v * ninv;
  uint32_t qh = __umulhi(q, n);
  uint32_t r;
  bool borrow = __builtin_usub_overflow((uint32_t)(v >> 32), qh, &r);
  return r + (borrow ? n : 0u);
}

// (m + s) mod n for m, s < n.
__device__ __forceinline__ uint32_t addmod32(uint32_t m, uint32_t s, uint32_t n) {
  uint32_t ns = n - s;
  uint32_t d = m - ns;
  return m < ns ? d + n : d;
}

// m^e mod n by left-to-right square-and-multiply on the unconverted message:
// the chain yields m^e 2^{-32(e-1)}, and one product with kc = 2^{32 e} mod n
// removes the factor.  EK selects a fixed chain (3, 5, 9, 17) or 0 for a
// chain over the bits of e.
template <int EK>
__device__ __forceinline__ uint32_t encrypt32(uint32_t m, uint32_t n, uint32_t ninv, uint32_t kc, uint64_t e,
                                              int ebits) {
  uint32_t x;
  if constexpr (EK == 3) {
    x = mont32(m, m, n, ninv);
    x = mont32(x, m, n, ninv);
  } else if constexpr (EK == 5) {
    x = mont32(m, m, n, ninv);
    x = mont32(x, x, n, ninv);
    x = mont32(x, m, n, ninv);
  } else if constexpr (EK == 9) {
    x = mont32(m, m, n, ninv);
    x = mont32(x, x, n, ninv);
    x = mont32(x, x, n, ninv);
    x = mont32(x, m, n, ninv);
  } else if constexpr (EK == 17) {
    x = mont32(m, m, n, ninv);
    x = mont32(x, x, n, ninv);
    x = mont32(x, x, n, ninv);
    x = mont32(x, x, n, ninv);
    x = mont32(x, m, n, ninv);
  } else {
    x = m;
    for (int b = ebits - 2; b >= 0; --b) {
      x = mont32(x, x, n, ninv);
      if ((e >> b) & 1) x = mont32(x, m, n, ninv);
    }
  }
  return mont32(x, kc, n, ninv);
}

// (c + 1) / (n + 1) correctly rounded, with rcp = RN(1/(n+1)) and den = n + 1
// (both exact integers below 2^33): q0 = a rcp is within 2 ulp, the remainder
// a - q0 den is exact, and one correction q0 + r rcp lands within 2^-52 ulp of
// a/den, which no rounding boundary approaches closer than ulp/2^33.
__device__ __forceinline__ double uniform32(uint32_t c, double den, double rcp) {
  double a = (double)(c + 1u);
  double q0 = a * rcp;
  double r = __builtin_fma(-q0, den, a);
  return __builtin_fma(r, rcp, q0);
}

// ---- 64-bit moduli from 32-bit limbs --------------------------------------

struct W128 {
  uint64_t lo, hi;
};

// a b + c in one v_mad_u64_u32.  Written out because the compiler
// reassociates a sum of two such products plus a 32-bit term into two
// products and a separate 64-bit add.
__device__ __forceinline__ uint64_t mad_u64_u32(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t r, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(carry) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Full product of x, y < 2^63.  The high words are below 2^31, so
// x1 y0 + x0 y1 + hi(x0 y0) < 2^64: three multiply-adds chain without a
// carry, and each 64-bit addend is a whole register pair.
__device__ __forceinline__ W128 mul63w(uint64_t x, uint64_t y) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  const uint64_t p00 = (uint64_t)x0 * y0;
  const uint64_t mid = mad_u64_u32(x1, y0, (uint64_t)x0 * y1 + (p00 >> 32));
  return {(mid << 32) | (uint32_t)p00, (uint64_t)x1 * y1 + (mid >> 32)};
}

// x^2 for x < 2^63: the cross term is one product with 2 x1 < 2^32.
__device__ __forceinline__ W128 sqr63w(uint64_t x) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint64_t p00 = (uint64_t)x0 * x0;
  // 2 x1 as one shift (the compiler otherwise forms it from both words)
  uint32_t x1d;
  asm("v_lshlrev_b32 %0, 1, %1" : "=v"(x1d) : "v"(x1));
  const uint64_t mid = (uint64_t)x0 * x1d + (p00 >> 32);
  return {(mid << 32) | (uint32_t)p00, (uint64_t)x1 * x1 + (mid >> 32)};
}

// High word of q n for n < 2^63: with h = hi(q0 n0), a = q1 n0 + h < 2^64
// and b = q0 n1 + lo(a) < 2^64, the high word is q1 n1 + hi(a) + hi(b).
__device__ __forceinline__ uint64_t mulhi_n63(uint64_t q, uint64_t n) {
  const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
  const uint32_t n0 = (uint32_t)n, n1 = (uint32_t)(n >> 32);
  const uint64_t a = (uint64_t)q1 * n0 + __umulhi(q0, n0);
  const uint64_t b = (uint64_t)q0 * n1 + (uint32_t)a;
  return (uint64_t)q1 * n1 + (a >> 32) + (b >> 32);
}

// v 2^{-64} mod n for v < n 2^64, n < 2^63 odd; ninv = n^{-1} mod 2^64.  The
// low words of v and q n cancel exactly, so the result is hi(v) - hi(q n)
// (+ n).
__device__ __forceinline__ uint64_t redc64(W128 v, uint64_t n, uint64_t ninv) {
  const uint64_t q = v.lo * ninv;
  const uint64_t qh = mulhi_n63(q, n);
  unsigned long r;
  bool borrow = __builtin_usubl_overflow(v.hi, qh, &r);
  return (uint64_t)r + (borrow ? n : 0ull);
}

// x y 2^{-64} mod n for x, y < n < 2^63.
__device__ __forceinline__ uint64_t mont64(uint64_t x, uint64_t y, uint64_t n, uint64_t ninv) {
  return redc64(mul63w(x, y), n, ninv);
}

// x^2 2^{-64} mod n for x < n < 2^63.
__device__ __forceinline__ uint64_t msqr64(uint64_t x, uint64_t n, uint64_t ninv) {
  return redc64(sqr63w(x), n, ninv);
}

// redc64 for a modulus that is the same in every lane of the wave (n and
// ninv are read from scalar registers; the compiler reads them from the
// first active lane if they sit in vector registers).  Same result as
// redc64, in fewer instructions: with q = lo(v) ninv mod 2^64 and
// h = hi(q0 n0), the middle column q1 n0 + h + q0 n1 can exceed 64 bits,
// and the multiply-add's carry-out supplies that bit, so
// hi(q n) = q1 n1 + (hi(middle) + carry 2^32) takes one multiply-add; the
// borrow of hi(v) - hi(q n) then selects the n that is added back (the
// compiler's form recomputes that borrow with a 64-bit compare).
//
// v0-v3 hold the intermediate register pairs (declared clobbered), and VCC
// carries each carry or borrow: gfx950 wants two wait states between a
// VALU write of VCC and a VALU read of it, hence the s_nop lines.
__device__ __forceinline__ uint64_t redc64_uniform(W128 v, uint64_t n, uint64_t ninv) {
  const uint64_t q = v.lo * ninv;
  const uint64_t h = __umulhi((uint32_t)q, (uint32_t)n);
  uint64_t r;
  asm("v_mad_u64_u32 v[0:1], vcc, %[q1], %[n0], %[h]\n\t"   // q1 n0 + h < 2^64
      "v_mad_u64_u32 v[0:1], vcc, %[q0], %[n1], v[0:1]\n\t"  // + q0 n1, carry-out in VCC
      "v_mov_b32 v2, v1\n\t"
      "s_nop 0\n\t"
      "v_cndmask_b32_e64 v3, 0, 1, vcc\n\t"                  // v[2:3] = hi(middle) + carry 2^32
      "v_mad_u64_u32 v[2:3], vcc, %[q1], %[n1], v[2:3]\n\t"  // hi(q n) < 2^64
      "v_sub_co_u32 v0, vcc, %[p0], v2\n\t"
      "s_nop 1\n\t"
      "v_subb_co_u32 v1, vcc, %[p1], v3, vcc\n\t"           // hi(v) - hi(q n), borrow in VCC
      "s_nop 1\n\t"
      "v_cndmask_b32 v2, 0, %[vn0], vcc\n\t"
      "v_cndmask_b32 v3, 0, %[vn1], vcc\n\t"
      "v_lshl_add_u64 %[r], v[0:1], 0, v[2:3]"               // + (borrow ? n : 0)
      : [r] "=v"(r)
      : [q0] "v"((uint32_t)q), [q1] "v"((uint32_t)(q >> 32)), [n0] "s"((uint32_t)n),
        [n1] "s"((uint32_t)(n >> 32)), [h] "v"(h), [p0] "v"((uint32_t)v.hi), [p1] "v"((uint32_t)(v.hi >> 32)),
        [vn0] "v"((uint32_t)n), [vn1] "v"((uint32_t)(n >> 32))
      : "v0", "v1", "v2", "v3", "vcc");
  return r;
}

__device__ __forceinline__ uint64_t mont64_uniform(uint64_t x, uint64_t y, uint64_t n, uint64_t ninv) {
  return redc64_uniform(mul63w(x, y), n, ninv);
}

__device__ __forceinline__ uint64_t msqr64_uniform(uint64_t x, uint64_t n, uint64_t ninv) {
  return redc64_uniform(sqr63w(x), n, ninv);
}

// (m + s) mod n for m, s < n < 2^63 (no overflow of the sum).
__device__ __forceinline__ uint64_t addmod64(uint64_t m, uint64_t s, uint64_t n) {
  uint64_t t = m + s;
  return t >= n ? t - n : t;
}

// v mod n for v < 4n (n < 2^63, so 2n fits 64 bits).
__device__ __forceinline__ uint64_t mod_below_4n(uint64_t v, uint64_t n) {
  const uint64_t n2 = n << 1;
  v = v >= n2 ? v - n2 : v;
  return v >= n ? v - n : v;
}

// m^e mod n (algorithm (9)) by a fixed chain for e = 3, 5, 9, 17, else by
// left-to-right squaring; n, ninv and kc = 2^{64 e} mod n are the same in
// every lane of the wave (one instance per tile).
template <int EK>
__device__ __forceinline__ uint64_t encrypt64(uint64_t m, uint64_t n, uint64_t ninv, uint64_t kc, uint64_t e,
                                              int ebits) {
  uint64_t x;
  if constexpr (EK == 3) {
    x = msqr64_uniform(m, n, ninv);
    x = mont64_uniform(x, m, n, ninv);
  } else if constexpr (EK == 5) {
    x = msqr64_uniform(m, n, ninv);
    x = msqr64_uniform(x, n, ninv);
    x = mont64_uniform(x, m, n, ninv);
  } else if constexpr (EK == 9) {
    x = msqr64_uniform(m, n, ninv);
    x = msqr64_uniform(x, n, ninv);
    x = msqr64_uniform(x, n, ninv);
    x = mont64_uniform(x, m, n, ninv);
  } else if constexpr (EK == 17) {
    x = msqr64_uniform(m, n, ninv);
    x = msqr64_uniform(x, n, ninv);
    x = msqr64_uniform(x, n, ninv);
    x = msqr64_uniform(x, n, ninv);
    x = mont64_uniform(x, m, n, ninv);
  } else {
    x = m;
    for (int b = ebits - 2; b >= 0; --b) {
      x = msqr64_uniform(x, n, ninv);
      if ((e >> b) & 1) x = mont64_uniform(x, m, n, ninv);
    }
  }
  return mont64_uniform(x, kc, n, ninv);
}

// Skip generator mod 2^61 - 1 (width 64): fold the 122-bit product.
__device__ __forceinline__ uint64_t mulmod_p61(uint64_t x, uint64_t y) {
  W128 t = mul63w(x, y);
  uint64_t lo = t.lo & kP64;
  uint64_t hi = (t.hi << 3) | (t.lo >> 61);
  uint64_t v = lo + hi;
  return v >= kP64 ? v - kP64 : v;
}

__device__ __forceinline__ uint64_t powmod_p61(uint64_t b, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mulmod_p61(r, b);
    b = mulmod_p61(b, b);
    e >>= 1;
  }
  return r;
}

// a^t mod (2^61 - 1) computed by the whole wave: lane b contributes
// pow2[b] = a^{2^b} when bit b of t is set, and the 64 factors are multiplied
// in a butterfly (six products per lane instead of up to 61 in sequence).
// Every lane receives the result.
__device__ __forceinline__ uint64_t wave_pow_p61(const uint64_t *pow2, uint64_t t, uint32_t lane) {
  uint64_t f = (lane < 61 && ((t >> lane) & 1)) ? pow2[lane] : 1ull;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = __shfl_xor((int)(uint32_t)f, d, 64);
    const uint32_t hi = __shfl_xor((int)(uint32_t)(f >> 32), d, 64);
    f = mulmod_p61(f, ((uint64_t)hi << 32) | lo);
  }
  return f;
}

// binary64(c + 1) / binary64(n + 1) correctly rounded, with den = RN(n + 1)
// and rcp = RN(1/den); c + 1 < 2^63 converts with one rounding.  The first
// correction makes the quotient faithful (within 1 ulp); from a faithful
// quotient and a correctly rounded reciprocal, one more remainder-and-
// correct step gives the correctly rounded quotient (Markstein), with five
// FP64 operations instead of the IEEE divide sequence.
__device__ __forceinline__ double uniform64(uint64_t c, double den, double rcp) {
  const double a = (double)(c + 1);
  const double q0 = a * rcp;
  const double q1 = __builtin_fma(__builtin_fma(-q0, den, a), rcp, q0);
  return __builtin_fma(__builtin_fma(-q1, den, a), rcp, q1);
}

// ---- instance set-up on the device (seeding) --------------------------------

__device__ __forceinline__ uint32_t inv32(uint32_t n) {  // n^{-1} mod 2^32, n odd (Newton)
  uint32_t x = n;
  for (int i = 0; i < 5; ++i) x *= 2u - n * x;
  return x;
}

__device__ __forceinline__ uint64_t inv64(uint64_t n) {  // n^{-1} mod 2^64, n odd (Newton)
  uint64_t x = n;
  for (int i = 0; i < 6; ++i) x *= 2ull - n * x;
  return x;
}

// Montgomery power: base and result in Montgomery form, one = R mod n.
__device__ __forceinline__ uint32_t mpow32(uint32_t b, uint64_t e, uint32_t one, uint32_t n, uint32_t ninv) {
  uint32_t r = one;
  while (e) {
    if (e & 1) r = mont32(r, b, n, ninv);
    b = mont32(b, b, n, ninv);
    e >>= 1;
  }
  return r;
}

__device__ __forceinline__ uint64_t mpow64(uint64_t b, uint64_t e, uint64_t one, uint64_t n, uint64_t ninv) {
  uint64_t r = one;
  while (e) {
    if (e & 1) r = mont64(r, b, n, ninv);
    b = mont64(b, b, n, ninv);
    e >>= 1;
  }
  return r;
}

// Deterministic Rabin-Miller for odd n in [2^31, 2^32): prime bases 2..11
// decide primality below 2^32 (Sec. IV).  No base is a multiple of n.
__device__ inline bool is_prime32_dev(uint32_t n) {
  const uint32_t ninv = inv32(n);
  const uint32_t one = 0u - n;  // 2^32 mod n (n > 2^31)
  uint32_t r2 = one;            // R^2 mod n: double R mod n 32 times
  for (int i = 0; i < 32; ++i) r2 = addmod32(r2, r2, n);
  const uint32_t mone = n - one;  // Montgomery form of n - 1
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  const uint32_t bases[5] = {2, 3, 5, 7, 11};
  for (int i = 0; i < 5; ++i) {
    uint32_t x = mpow32(mont32(bases[i], r2, n, ninv), d, one, n, ninv);
    if (x == one || x == mone) continue;
    bool witness = true;
    for (int j = 1; j < s; ++j) {
      x = mont32(x, x, n, ninv);
      if (x == mone) {
        witness = false;
        break;
      }
    }
    if (witness) return false;
  }
  return true;
}

// Deterministic Rabin-Miller for odd n in [2^62, 2^63): the twelve prime
// bases 2..37 decide primality below 2^64 (Sec. IV).
__device__ inline bool is_prime64_dev(uint64_t n) {
  const uint64_t ninv = inv64(n);
  uint64_t one = 0ull - n;  // 2^64 - n, then reduce: 2^64 mod n
  while (one >= n) one -= n;
  uint64_t r2 = one;
  for (int i = 0; i < 64; ++i) r2 = addmod64(r2, r2, n);
  const uint64_t mone = n - one;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  const uint32_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (int i = 0; i < 12; ++i) {
    uint64_t x = mpow64(mont64(bases[i], r2, n, ninv), d, one, n, ninv);
    if (x == one || x == mone) continue;
    bool witness = true;
    for (int j = 1; j < s; ++j) {
      x = mont64(x, x, n, ninv);
      if (x == mone) {
        witness = false;
        break;
      }
    }
    if (witness) return false;
  }
  return true;
}

// j-th output (j = 0, 1, ...) of the SplitMix64 stream started at `seed`
// (Steele, Lea and Flood, 2014): the state after j+1 steps, finalised.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---- wave helpers ---------------------------------------------------------

// Load of a record that no kernel writes while this one runs, at an address
// that is the same in every lane: through the constant address space, so that
// the compiler reads it with scalar loads into SGPRs and the arithmetic on it
// runs on the scalar unit instead of in every lane.
template <typename T>
__device__ __forceinline__ T const_load(const T *p) {
  static_assert(sizeof(T) % 8 == 0, "records of whole 64-bit words");
  using CP = const __attribute__((address_space(4))) uint64_t *;
  const CP q = (CP)p;
  T out;
  uint64_t *o = reinterpret_cast<uint64_t *>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 8); ++i) o[i] = q[i];
  return out;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
  uint32_t lo = __shfl_up((int)(uint32_t)v, d, 64);
  uint32_t hi = __shfl_up((int)(uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((int)(uint32_t)v, src, 64);
  uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  uint32_t lo = __shfl_xor((int)(uint32_t)v, mask, 64);
  uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Sum of v over the 64 lanes of the wave, mod n (v < n < 2^63); every lane
// receives it.
__device__ __forceinline__ uint64_t wave_sum_mod(uint64_t v, uint64_t n) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t t = v + shfl_xor_u64(v, d);
    v = t >= n ? t - n : t;
  }
  return v;
}

// Exclusive prefix sum of v over the lanes of the wave, mod n (v < n < 2^63).
__device__ __forceinline__ uint64_t wave_exclusive_mod(uint64_t v, uint64_t n, uint32_t lane) {
  uint64_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t u = shfl_up_u64(incl, d);
    if ((int)lane >= d) {
      const uint64_t t = incl + u;
      incl = t >= n ? t - n : t;
    }
  }
  return incl >= v ? incl - v : incl + (n - v);
}

// Orders this wave's LDS accesses across lanes (all lanes of one wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace dev
}  // namespace phprng
