// Wave-level complex transforms with the positive exponent for gfx950: one
// wave (or half a wave) holds a whole transform of N = 16 P points, 16 per
// lane, P in {32, 64}.  With n = l + P m and k = k_a + 16 (k_b1 + 16 q):
//   1. lane l: 16-point transform over m in registers, times w_N^{l k_a};
//   2. one transpose through the wave's own LDS area (row stride P + 1);
//   3. lane t = (k_a, l_a), k_a = t / R, l_a = t % R, R = P / 16: 16-point
//      transform over l_b of the points l = l_a + R l_b, times w_P^{l_a k_b1};
//   4. R-point transform across the R lanes of each k_a group with DPP moves
//      (radix 2 per lane bit, R = 2 or 4).
// No workgroup barrier is involved: the LDS area belongs to the wave.  The
// twiddles of steps 1 and 3 are powers of one root per lane (15 products
// each; about 15 ulp of accumulated rounding, far below the transform's own
// error), so a lane loads two roots instead of thirty.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace phprng {
namespace wf {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmulw(double2 a, double2 w) {
  return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
__device__ __forceinline__ double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }

// 4-point transform, positive exponent, in place, natural order.
__device__ __forceinline__ void dft4(double2 &a0, double2 &a1, double2 &a2, double2 &a3) {
  const double2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3), b3 = mul_i(csub(a1, a3));
  a0 = cadd(b0, b2);
  a1 = cadd(b1, b3);
  a2 = csub(b0, b2);
  a3 = csub(b1, b3);
}

// exp(2 pi i j / 16) for the products inside a 16-point transform.
constexpr double kC1 = 0.9238795325112867561281831893967882868224;  // cos(pi/8)
constexpr double kS1 = 0.3826834323650897717284599840303988667613;  // sin(pi/8)
constexpr double kR2 = 0.7071067811865475244008443621048490392848;  // sqrt(2)/2

// 16-point transform, positive exponent, natural-order output: with
// m = m0 + 4 m1 and k = k1 + 4 k0, four 4-point transforms over m1, the
// products w16^{m0 k1}, four 4-point transforms over m0.
__device__ __forceinline__ void dft16(double2 (&v)[16]) {
#pragma unroll
  for (int m0 = 0; m0 < 4; ++m0) dft4(v[m0], v[m0 + 4], v[m0 + 8], v[m0 + 12]);
  // v[m0 + 4 k1] *= w16^{m0 k1}
  v[5] = cmulw(v[5], make_double2(kC1, kS1));     // w^1
  v[9] = cmulw(v[9], make_double2(kR2, kR2));     // w^2
  v[13] = cmulw(v[13], make_double2(kS1, kC1));   // w^3
  v[6] = cmulw(v[6], make_double2(kR2, kR2));     // w^2
  v[10] = mul_i(v[10]);                           // w^4
  v[14] = cmulw(v[14], make_double2(-kR2, kR2));  // w^6
  v[7] = cmulw(v[7], make_double2(kS1, kC1));     // w^3
  v[11] = cmulw(v[11], make_double2(-kR2, kR2));  // w^6
  v[15] = cmulw(v[15], make_double2(-kC1, -kS1)); // w^9
  double2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    double2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4(a0, a1, a2, a3);
    o[k1] = a0;
    o[k1 + 4] = a1;
    o[k1 + 8] = a2;
    o[k1 + 12] = a3;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}

// exp(2 pi i j / 16), j = 0 .. 8.
__device__ __forceinline__ double2 w16(int j) {
  switch (j) {
    case 0: return make_double2(1.0, 0.0);
    case 1: return make_double2(kC1, kS1);
    case 2: return make_double2(kR2, kR2);
    case 3: return make_double2(kS1, kC1);
    case 4: return make_double2(0.0, 1.0);
    case 5: return make_double2(-kS1, kC1);
    case 6: return make_double2(-kR2, kR2);
    case 7: return make_double2(-kC1, kS1);
    default: return make_double2(-1.0, 0.0);
  }
}

// Lane exchange inside groups of 4 lanes (DPP quad permutations).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]

template <int CTRL>
__device__ __forceinline__ double2 dpp_c(double2 a) {
  return make_double2(dpp_d<CTRL>(a.x), dpp_d<CTRL>(a.y));
}

// Steps 1 and 3-4 of the wave transform below (the parts outside the
// transpose).  wave_before: the 16-point transform over m and the products
// w_N^{l k_a}.  wave_after: for lane t = (k_a, l_a), the 16-point transform
// over l_b, the products w_P^{l_a k_b1}, and the R-point transform across the
// lanes of the k_a group.
template <int P>
__device__ __forceinline__ void wave_before(double2 (&v)[16], const double2 *__restrict__ w1024, uint32_t l) {
  constexpr int N = 16 * P;
  static_assert(P == 32 || P == 64, "wave transform sizes");
  dft16(v);
  // w_N^{l ka} as powers of one loaded root (15 products, no further loads)
  const double2 wl = w1024[l * (1024 / N)];
  double2 wk = wl;
#pragma unroll
  for (int ka = 1; ka < 16; ++ka) {
    v[ka] = cmulw(v[ka], wk);
    wk = cmulw(wk, wl);
  }
}

template <int P>
__device__ __forceinline__ void wave_after(double2 (&v)[16], const double2 *__restrict__ w1024, uint32_t la) {
  constexpr int R = P / 16;
  dft16(v);
  const double2 wa = w1024[la * (1024 / P)];
  double2 wb = wa;
#pragma unroll
  for (int kb = 1; kb < 16; ++kb) {
    v[kb] = cmulw(v[kb], wb);
    wb = cmulw(wb, wa);
  }
  if constexpr (R == 2) {
    // lane pair (a = 0, 1): X_0 = C_0 + C_1 on a = 0, X_1 = C_0 - C_1 on a = 1
    const bool hi = (la & 1) != 0;
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
      const double2 o = dpp_c<kQuadXor1>(v[kb]);
      v[kb] = hi ? csub(o, v[kb]) : cadd(v[kb], o);
    }
  } else {
    // a = a0 + 2 a1.  Stage 1 (partner a ^ 2): a1 = 0 keeps C_a0 + C_a0+2,
    // a1 = 1 keeps w4^{a0} (C_a0 - C_a0+2).  Stage 2 (partner a ^ 1): a0 = 0
    // keeps D_0 + D_1 = X_{a1}, a0 = 1 keeps D_0 - D_1 = X_{a1 + 2}.
    const bool a0 = (la & 1) != 0, a1 = (la & 2) != 0;
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
      const double2 o = dpp_c<kQuadXor2>(v[kb]);
      double2 d = a1 ? csub(o, v[kb]) : cadd(v[kb], o);
      if (a1 && a0) d = mul_i(d);
      const double2 o2 = dpp_c<kQuadXor1>(d);
      v[kb] = a0 ? csub(o2, d) : cadd(d, o2);
    }
  }
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The transform of N = 16 P points held by the P lanes [base, base + P) of a
// wave (lane l = threadIdx.x % 64 - base): on entry v[m] = x[l + P m]; on exit
// v[k_b1] = X[k_a + 16 k_b1 + 256 q] for lane t = l with k_a = t / R and q the
// lane's output index in its group (q = t % 2 for R = 2; for R = 4 the two
// bits of t % 4 swapped).  lds: this lane group's area of 16 (P + 1) double2.
// w1024[j] = exp(2 pi i j / 1024).
template <int P>
__device__ __forceinline__ void wave_fft(double2 (&v)[16], double2 *lds, const double2 *__restrict__ w1024,
                                         uint32_t l) {
  constexpr int R = P / 16, S = P + 1;
  wave_before<P>(v, w1024, l);
  // transpose: row k_a, column l
#pragma unroll
  for (int ka = 0; ka < 16; ++ka) lds[ka * S + l] = v[ka];
  wave_lds_fence();
  const uint32_t ka = l / R, la = l % R;
#pragma unroll
  for (int lb = 0; lb < 16; ++lb) v[lb] = lds[ka * S + la + R * lb];
  wave_after<P>(v, w1024, la);
}

// wave_fft with the transpose taken in two rounds through an area of doubles,
// real parts then imaginary parts: half the LDS, and no more live registers
// (the real parts of v are dead once written; the imaginary parts are read
// in their own round).  lds: this lane group's area of 16 (P + 1) doubles.
template <int P>
__device__ __forceinline__ void wave_fft_split(double2 (&v)[16], double *lds, const double2 *__restrict__ w1024,
                                               uint32_t l) {
  constexpr int R = P / 16, S = P + 1;
  wave_before<P>(v, w1024, l);
  const uint32_t ka = l / R, la = l % R;
  double re[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[k * S + l] = v[k].x;
  wave_lds_fence();
#pragma unroll
  for (int lb = 0; lb < 16; ++lb) re[lb] = lds[ka * S + la + R * lb];
  wave_lds_fence();
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[k * S + l] = v[k].y;
  wave_lds_fence();
#pragma unroll
  for (int lb = 0; lb < 16; ++lb) v[lb] = make_double2(re[lb], lds[ka * S + la + R * lb]);
  wave_after<P>(v, w1024, la);
}

// Output index q of lane t within its group (see wave_fft).
template <int P>
__device__ __forceinline__ uint32_t wave_fft_q(uint32_t t) {
  if constexpr (P == 32) return t & 1;
  return ((t & 1) << 1) | ((t >> 1) & 1);
}

}  // namespace wf
}  // namespace phprng
