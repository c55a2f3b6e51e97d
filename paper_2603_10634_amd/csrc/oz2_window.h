// Decision window of the accurate mode's scale exponents (Section III-E),
// shared by the scale kernels and a host build used by the tests.
//
// The bound product Abar Bbar has non-negative terms and runs on the FP8
// MFMA, so each computed line maximum r' differs from the exact maximum r.
// The window below is derived from this stated worst case of the FP8 MFMA's
// accumulation (W):
//
//  (W1) products are summed in groups of 8 consecutive k; inside a group every
//       product other than the largest, g, may be replaced by any value within
//       2^-13 ufp(g) <= 2^-13 g of it (truncation or rounding of the aligned
//       products, either direction);
//  (W2) every addition of a group sum into the FP32 accumulator is faithfully
//       rounded: its error is below one ulp of the result, <= 2^-23 of it, in
//       either direction.
//
// (The measured behaviour of v_mfma_f32_32x32x64_f8f6f4 is narrower: the
// products are truncated toward zero inside a group and the accumulator
// rounds up at most once per instruction.)  When the k range is split into
// `parts` ranges whose FP32 sums are added afterwards (each addition rounded
// to nearest, within (W2)), every group sum passes through at most
// ceil(k/8) + parts - 1 additions.  For one output c = sum_h x_h with x_h >= 0
// and Q = ceil(k/8) + parts - 1, a group sum s changes by less than
// 7 2^-13 g <= 7 2^-13 s by (W1), and at most Q faithful additions multiply
// it by at most (1 +- 2^-23)^Q, so with e1 = 7 2^-13, u = 2^-23:
//     c (1 - gu) <= c' <= c (1 + go),
//     gu = e1 + Q u,   go = e1 + 1.02 Q u   (for Q u <= 2^-7, i.e. k <= 2^18
//     with up to 2^14 parts; (1 + e1)(1 + u)^Q <= (1 + e1)(1 + 1.004 Q u)
//     <= 1 + e1 + 1.02 Q u).
// The maximum over a line inherits both bounds (r' >= c'_max >= r (1 - gu),
// r' <= max_j c_j (1 + go) = r (1 + go)), so
//     r'/(1 + go) <= r <= r'/(1 - gu).
// The library's window doubles both deviations:
//     lo = r'/(1 + 2 go),  hi = r'/(1 - 2 gu),
// each computed in double and widened by 2^-50 for its own rounding.  A line
// whose whole window [lo, hi] gives one exponent has that exponent for its
// exact maximum (the rule is monotone in r); any other line is recomputed
// exactly.  A wider window costs only more exact recomputations.
#pragma once

#include <math.h>
#include <stdint.h>

#ifndef OZ2_HD
#if defined(__HIPCC__)
#define OZ2_HD __host__ __device__
#else
#define OZ2_HD
#endif
#endif

namespace oz2 {

// Relative deviations of (W) for a k extent of kp summed in `parts` ranges:
// c (1 - gu) <= c' <= c (1 + go).
OZ2_HD inline void bound_deviation(int64_t kp, int parts, double *gu, double *go) {
  const double Q = (double)((kp + 7) / 8 + parts - 1);
  const double e1 = 7.0 * 0x1p-13;
  *gu = e1 + Q * 0x1p-23;
  *go = e1 + 1.02 * Q * 0x1p-23;
}

// The library's window [lo, hi] for the exact line maximum, given the
// computed one r' (twice the deviations of (W)).
OZ2_HD inline void bound_window(double rp, int64_t kp, int parts, double *lo, double *hi) {
  double gu, go;
  bound_deviation(kp, parts, &gu, &go);
  *lo = rp / (1.0 + 2.0 * go) * (1.0 - 0x1p-50);
  *hi = rp / (1.0 - 2.0 * gu) * (1.0 + 0x1p-50);
}

// max{e : x 2^(2e+1) <= D} for a double x > 0, where D is the largest double
// not above P - 1 (so for a double y, y <= P - 1 iff y <= D).
OZ2_HD inline int exponent_rule(double x, double D) {
  int ex, eD;
  const double mx = frexp(x, &ex);
  const double mD = frexp(D, &eD);
  const int d = eD - ex - 1 - (mx > mD ? 1 : 0);
  return d >= 0 ? d / 2 : -((-d + 1) / 2);  // floor(d / 2)
}

// Scale exponents of the two ends of the window of a computed maximum rp > 0:
// equal values settle the line, different ones send it to the exact fix-up.
OZ2_HD inline void window_exponents(double rp, int64_t kp, int parts, double D,
                                    int *e_small, int *e_large) {
  double lo, hi;
  bound_window(rp, kp, parts, &lo, &hi);
  *e_small = exponent_rule(hi, D);
  *e_large = exponent_rule(lo, D);
}

}  // namespace oz2
