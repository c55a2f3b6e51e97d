// Device helpers shared by the kernels: exact bit-level handling of FP64
// inputs and of the FP8 E4M3 (OCP E4M3FN: bias 7, max 448, no infinities)
// encodings used for the bound operands and the residue digits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oz2 {

// Split a finite double into |x| = mant * 2^q with mant < 2^53 (an integer).
__device__ __forceinline__ void split_double(uint64_t bits, uint64_t &mant, int &q) {
  int ex = (int)((bits >> 52) & 0x7FF);
  mant = bits & ((1ull << 52) - 1);
  if (ex == 0) {
    q = -1074;
  } else {
    mant |= 1ull << 52;
    q = ex - 1075;
  }
}

// floor(log2 |x|) of a finite nonzero double given its bits.
__device__ __forceinline__ int ufp_exponent(uint64_t bits) {
  int ex = (int)((bits >> 52) & 0x7FF);
  if (ex != 0) return ex - 1023;
  uint64_t man = bits & ((1ull << 52) - 1);
  return (63 - __clzll((long long)man)) - 1074;
}

__device__ __forceinline__ bool is_nonfinite(uint64_t bits) {
  return ((bits >> 52) & 0x7FF) == 0x7FF;
}

// E4M3 code of the smallest E4M3 value >= |x| * 2^sh for a finite double
// (given as bits) whose scaled magnitude is below 2^8 + 1 (Section III-E cast
// of mu'|A| in round-up mode).  Exact integer arithmetic throughout.
__device__ __forceinline__ uint32_t e4m3_round_up(uint64_t bits, int sh) {
  uint64_t mant;
  int q;
  split_double(bits & 0x7FFFFFFFFFFFFFFFull, mant, q);
  if (mant == 0) return 0u;
  int bl = 64 - __clzll((long long)mant);  // bit length of mant
  int bexp = bl - 1 + q + sh;              // floor(log2 of the scaled value)
  if (bexp >= -6) {
    // normal: 4 significant bits, rounded up
    int drop = bl - 4;                     // >= 0 since mant of a normal double has 53 bits
    uint64_t Q;
    if (drop > 0) {
      Q = mant >> drop;
      if (mant & ((1ull << drop) - 1)) Q += 1;
    } else {
      Q = mant << (-drop);
    }
    if (Q == 16) {
      Q = 8;
      bexp += 1;
    }
    return (uint32_t)(((bexp + 7) << 3) | (int)(Q - 8));
  }
  // subnormal grid 2^-9: Q = ceil(value / 2^-9) in [1, 8]; Q = 8 is the code
  // of 2^-6, the smallest normal
  // value / 2^-9 = mant * 2^s2; s2 <= 3 - bitlength(mant), so s2 > 0 only
  // for the few-bit mantissas of subnormal doubles
  int s2 = q + sh + 9;
  uint64_t Q;
  if (s2 >= 0) {
    Q = mant << s2;
  } else if (-s2 >= 64) {
    Q = 1;
  } else {
    int r = -s2;
    Q = mant >> r;
    if (mant & ((1ull << r) - 1)) Q += 1;
  }
  return (uint32_t)Q;
}

// E4M3 code of a small integer d with |d| <= 16 (exact in the format).
__device__ __forceinline__ uint32_t e4m3_of_small_int(int d) {
  uint32_t a = (uint32_t)(d < 0 ? -d : d);
  if (a == 0) return 0u;
  int e = 31 - __clz((int)a);               // 0..4
  uint32_t man = ((a << 3) >> e) - 8u;      // 3 mantissa bits, exact
  uint32_t code = ((uint32_t)(e + 7) << 3) | man;
  return d < 0 ? (code | 0x80u) : code;
}

// 2^9 x the value of a non-negative E4M3 code (sign bit clear): an integer
// below 2^18.  Subnormals (exponent field 0) are m 2^-9, normals
// (8 + m) 2^(e - 10).
__device__ __forceinline__ uint32_t e4m3_q9(uint32_t code) {
  const uint32_t ex = code >> 3, man = code & 7u;
  return ex ? (8u + man) << (ex - 1u) : man;
}

}  // namespace oz2
