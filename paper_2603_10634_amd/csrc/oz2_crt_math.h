// Exact integer arithmetic of the CRT reconstruction (eq. CRT_finalreduction)
// and of the one rounding of the inverse scaling (eq. inversescaling): the
// reduction of S = sum_l w_l u_l modulo P to C' and RN(C' 2^-t).  Host and
// device functions alike, so that the host can check them against exact
// integer results; the CRT kernel is their only device caller.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "oz2_internal.h"

namespace oz2 {

// Bits [pos, pos + 64) of a little-endian limb array (zeros beyond the end).
template <int L>
__host__ __device__ __forceinline__ uint64_t window64(const uint32_t (&x)[L], int pos) {
  const int w = pos >> 5, b = pos & 31;
  uint32_t x0 = 0, x1 = 0, x2 = 0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    x0 = (q == w) ? x[q] : x0;
    x1 = (q == w + 1) ? x[q] : x1;
    x2 = (q == w + 2) ? x[q] : x2;
  }
  const uint64_t lo = (uint64_t)x0 | ((uint64_t)x1 << 32);
  if (b == 0) return lo;
  return (lo >> b) | ((uint64_t)x2 << (64 - b));
}

// True if any bit below position pos is set.
template <int L>
__host__ __device__ __forceinline__ bool any_below(const uint32_t (&x)[L], int pos) {
  uint32_t acc = 0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int lo = 32 * q;
    uint32_t mask;
    if (pos >= lo + 32)
      mask = 0xFFFFFFFFu;
    else if (pos <= lo)
      mask = 0u;
    else
      mask = (1u << (pos - lo)) - 1u;
    acc |= x[q] & mask;
  }
  return acc != 0;
}

// RN-even of X 2^-t for a non-negative integer X (L limbs), bit by bit: the
// 53 kept bits, the round bit and the sticky bits at the position the result's
// exponent gives, gradual underflow included.
template <int L>
__host__ __device__ __forceinline__ double scaled_rn_exact(const uint32_t (&X)[L], int t) {
  int hb = -1;
#pragma unroll
  for (int q = 0; q < L; ++q)
    if (X[q]) hb = 32 * q + 31 - __builtin_clz(X[q]);
  if (hb < 0) return 0.0;
  // position of the last kept bit: 53 significant bits, but not below 2^-1074
  int lsb = hb - 52;
  if (t - 1074 > lsb) lsb = t - 1074;
  if (lsb < 0) lsb = 0;
  uint64_t Q = window64<L>(X, lsb) & ((1ull << 54) - 1);  // <= 53 bits are set
  if (lsb > 0) {
    const bool rbit = (window64<L>(X, lsb - 1) & 1ull) != 0;
    const bool sticky = any_below<L>(X, lsb - 1);
    if (rbit && (sticky || (Q & 1ull))) Q += 1;
  }
  return ldexp((double)Q, lsb - t);
}

// RN-even of X 2^-t for a non-negative integer X (L limbs).  With h the top
// nonzero limb and c the leading zeros of X[h], the 64 bits below the leading
// bit, U = floor(X 2^(c + 32 - 32 h)) (limbs h, h - 1, h - 2 shifted left by
// c), hold the 53 kept bits and the round bit of X; any bit of X below U is
// folded into U's lowest bit, which lies below the round bit, so RN(U') =
// RN(X 2^(c + 32 - 32 h)).  RN(U') is one fused multiply-add of two exact
// halves, and scaling it by 2^(32 h - 32 - c - t) is exact when the result is
// normal (it overflows to infinity exactly when RN(X 2^-t) does).  A result
// below 2^-1022 takes the bit-by-bit rounding, whose position depends on the
// exponent.
template <int L>
__host__ __device__ __forceinline__ double scaled_rn(const uint32_t (&X)[L], int t) {
  int h = -1;
#pragma unroll
  for (int q = 0; q < L; ++q)
    if (X[q]) h = q;
  if (h < 0) return 0.0;
  uint32_t T2 = 0, T1 = 0, T0 = 0, below = 0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    T2 = (q == h) ? X[q] : T2;
    T1 = (q == h - 1) ? X[q] : T1;
    T0 = (q == h - 2) ? X[q] : T0;
    below |= (q < h - 2) ? X[q] : 0u;
  }
  const int c = __builtin_clz(T2);
  if (32 * h + 31 - c - t < -1022) return scaled_rn_exact<L>(X, t);
  const uint64_t lo = (((uint64_t)T1 << 32) | T0) << c;
  const uint32_t u2 = (T2 << c) | ((T1 >> 1) >> (31 - c));  // no shift by 32 for c = 0
  const uint32_t u1 = (uint32_t)(lo >> 32) | ((below | (uint32_t)lo) != 0u ? 1u : 0u);
  const double u = fma((double)u2, 0x1p32, (double)u1);
  return ldexp(u, 32 * h - 32 - c - t);
}

// D = sum_q r[q] 2^(32 q) for integers |r[q]| < 2^49 and |D| < 2^(32 L): its
// magnitude in 32-bit limbs, its sign, and an estimate d of D.  The carries
// are exact (x - 2^32 floor(x 2^-32) by one fused multiply-add); the last one
// is -1 or 0, the sign.  d is Horner's rule over the normalised limbs, whose
// partial values are floor(D 2^-32q): |d - D| <= 2^-53 (L |D| + 2^(32 L - 31)).
template <int L>
__host__ __device__ __forceinline__ bool crt_normalize(const double (&r)[L], uint32_t (&mag)[L],
                                              double &d) {
  double lo[L];
  double c = 0.0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const double x = r[q] + c;
    const double hi = floor(x * 0x1p-32);
    lo[q] = fma(-hi, 0x1p32, x);
    c = hi;
  }
  d = c;
#pragma unroll
  for (int q = L - 1; q >= 0; --q) d = fma(d, 0x1p32, lo[q]);
  const bool neg = c < 0.0;
  // |D| = 2^(32 L) - sum lo[q] 2^(32 q) when D < 0: a borrow chain from 0
  uint32_t borrow = 0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const uint32_t u = (uint32_t)lo[q];
    const uint32_t v = 0u - u - borrow;
    borrow = (u | borrow) != 0u ? 1u : 0u;
    mag[q] = neg ? v : u;
  }
  return neg;
}

// x > y for L-limb numbers.
template <int L>
__host__ __device__ __forceinline__ bool limbs_greater(const uint32_t (&x)[L], const uint32_t *y) {
  bool gt = false, decided = false;
#pragma unroll
  for (int q = L - 1; q >= 0; --q) {
    if (!decided && x[q] != y[q]) {
      gt = x[q] > y[q];
      decided = true;
    }
  }
  return gt;
}

// C' = S mods P (the representative in [-floor(P/2), P - 1 - floor(P/2)])
// for S = sum_q acc[q] 2^(32 q), |acc[q]| < 2^47: its magnitude in mag and
// its sign as the result.  P has L <= 10 limbs and |S| < 2^15 P.
//   Q = rint(S / P) from S by Horner's rule times 1/P: the rounding errors
//     add up to less than 2^-53 (L |S| / P + 2^16) + 2^-51 |S| / P < 2^-33
//     in S / P, so Q is the nearest integer, or one off when S / P is
//     within 2^-33 of a half-integer;
//   D = S - Q P limb by limb, exactly (|Q P_q| < 2^47);
//   if the estimate of D is at most crt_fast = P (1/2 - 2^-40) - 2 in
//   magnitude, D is C' (the estimate is within 2^-53 (L |D| + 2 P) < 2^-49 P
//   of D, so |D| < floor(P/2) - 1); otherwise D is compared with the range
//   exactly and moved by P when it lies outside.
template <int L>
__host__ __device__ __forceinline__ bool crt_reduce(const double (&acc)[L], const Tables *__restrict__ tab,
                                           uint32_t (&mag)[L]) {
  double sa = acc[L - 1];
#pragma unroll
  for (int q = L - 2; q >= 0; --q) sa = fma(sa, 0x1p32, acc[q]);
  const double Q = rint(sa * tab->inv_P_d);
  double r[L];
#pragma unroll
  for (int q = 0; q < L; ++q) r[q] = fma(-Q, tab->Pdl[q], acc[q]);
  double d;
  bool neg = crt_normalize<L>(r, mag, d);
  if (fabs(d) > tab->crt_fast) {
    // D >= 0 must not exceed P - 1 - floor(P/2), D < 0 not -floor(P/2)
    if (limbs_greater<L>(mag, neg ? tab->half : tab->top)) {
#pragma unroll
      for (int q = 0; q < L; ++q) r[q] += neg ? tab->Pdl[q] : -tab->Pdl[q];
      neg = crt_normalize<L>(r, mag, d);
    }
  }
  return neg;
}

}  // namespace oz2
