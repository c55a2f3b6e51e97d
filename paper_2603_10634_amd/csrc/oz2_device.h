// Device helpers shared by the kernels: exact handling of FP64 inputs and of
// the FP8 E4M3 (OCP E4M3FN: bias 7, max 448, no infinities) encodings used
// for the bound operands and the residue digits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oz2 {

// floor(log2 |x|) of a finite nonzero double given its bits.
__device__ __forceinline__ int ufp_exponent(uint64_t bits) {
  int ex = (int)((bits >> 52) & 0x7FF);
  if (ex != 0) return ex - 1023;
  uint64_t man = bits & ((1ull << 52) - 1);
  return (63 - __clzll((long long)man)) - 1074;
}

// E4M3 code of the smallest E4M3 value >= |a| 2^sh for a finite nonzero
// double a whose scaled magnitude y = |a| 2^sh is below 2^8 + 1 (Section
// III-E cast of mu'|A| in round-up mode).  With e = max(floor(log2 y), -6)
// the E4M3 values near y are spaced 2^(e - 3) (below 2^-6 the subnormal
// spacing 2^-9 = 2^(-6 - 3)), so the result is Q 2^(e - 3) with
// Q = ceil(y 2^(3 - e)) in [1, 16], and its code is 8 (e + 7) + Q - 8:
// Q = 16 carries into the next binade's code, and at e = -6 the codes 1..8
// are the subnormals and the smallest normal.  The scaling by
// 2^(sh + 3 - e) is exact unless its result falls below 2^-1022, where y is
// far below one spacing and Q = 1; hence the maximum with one.
__device__ __forceinline__ uint32_t e4m3_round_up(double a, int sh) {
  const int fl = __builtin_amdgcn_frexp_exp(a) - 1 + sh;  // floor(log2 y)
  const int e = fl > -6 ? fl : -6;
  const double Q = fmax(ceil(ldexp(fabs(a), sh + 3 - e)), 1.0);
  return (uint32_t)(8 * e + 48 + (int)Q);
}

// 2^9 x the value of a non-negative E4M3 code (sign bit clear): an integer
// below 2^18.  Subnormals (exponent field 0) are m 2^-9, normals
// (8 + m) 2^(e - 10).
__device__ __forceinline__ uint32_t e4m3_q9(uint32_t code) {
  const uint32_t ex = code >> 3, man = code & 7u;
  return ex ? (8u + man) << (ex - 1u) : man;
}

}  // namespace oz2
