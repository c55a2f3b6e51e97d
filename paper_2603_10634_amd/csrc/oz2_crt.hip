// Chinese-remainder reconstruction and inverse scaling (eqs.
// CRT_finalreduction, inversescaling), fused with alpha/beta.
//
// Per output entry (i, j): the residues u_l = C'_l (symmetric range) from the
// int16 planes; S = sum_l w_l u_l in 32-bit limbs held as exact FP64
// integers; C' = S mods P, the representative in [-floor(P/2),
// P - 1 - floor(P/2)], which is the product itself by condition (3).  Then
// Chat = C' 2^-(log2 mu_i + log2 nu_j) rounded once to nearest-even,
// including gradual underflow, directly from the integer: no intermediate
// floating-point rounding.  C = RN(alpha Chat) (+ RN(beta C_in)).
#include <string.h>

#include "oz2_internal.h"

namespace oz2 {

namespace {

// Bits [pos, pos + 64) of a little-endian limb array (zeros beyond the end).
template <int L>
__device__ __forceinline__ uint64_t window64(const uint32_t (&x)[L], int pos) {
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
__device__ __forceinline__ bool any_below(const uint32_t (&x)[L], int pos) {
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

// RN-even of X 2^-t for a non-negative integer X (L limbs).
template <int L>
__device__ __forceinline__ double scaled_rn(const uint32_t (&X)[L], int t) {
  int hb = -1;
#pragma unroll
  for (int q = 0; q < L; ++q)
    if (X[q]) hb = 32 * q + 31 - __clz((int)X[q]);
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

// D = sum_q r[q] 2^(32 q) for integers |r[q]| < 2^49 and |D| < 2^(32 L): its
// magnitude in 32-bit limbs, its sign, and an estimate d of D.  The carries
// are exact (x - 2^32 floor(x 2^-32) by one fused multiply-add); the last one
// is -1 or 0, the sign.  d is Horner's rule over the normalised limbs, whose
// partial values are floor(D 2^-32q): |d - D| <= 2^-53 (L |D| + 2^(32 L - 31)).
template <int L>
__device__ __forceinline__ bool crt_normalize(const double (&r)[L], uint32_t (&mag)[L],
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
__device__ __forceinline__ bool limbs_greater(const uint32_t (&x)[L], const uint32_t *y) {
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
__device__ __forceinline__ bool crt_reduce(const double (&acc)[L], const Tables *__restrict__ tab,
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

// NF > 0: the number of moduli is the compile-time NF (no per-modulus
// branches); NF = 0: N at run time.
template <int L, int NF>
__device__ __forceinline__ void crt_entry(const int16_t *__restrict__ planes,
                                          const int32_t *__restrict__ shift,
                                          const uint32_t *__restrict__ flags,
                                          const Tables *__restrict__ tab, int N, int64_t m,
                                          int64_t mp, int64_t np, int64_t lineB, double alpha,
                                          double beta, double *__restrict__ C, int64_t ldc,
                                          int64_t i, int64_t j) {
  if (i >= m) return;
  const bool bad = ((flags[i] | flags[lineB + j]) & kNonFinite) != 0;
  double chat;
  if (bad) {
    chat = __longlong_as_double(0x7FF8000000000000ll);
  } else {
    // S = sum_l w_l u_l over the stored residues u_l (C'_l in the symmetric
    // range; any representative changes S by a multiple of P), accumulated
    // per 32-bit limb in FP64 (full rate on this GPU, unlike 64-bit integer
    // multiply-adds): |w_l,q u_l| < 2^42, so every limb sum of at most
    // kMaxN terms is an exact integer below 2^47
    double acc[L];
#pragma unroll
    for (int q = 0; q < L; ++q) acc[q] = 0.0;
    const int16_t *pl = planes + j * mp + i;
    const int64_t pstride = mp * np;
    // all N residues are requested before the first is used
    const int NN = NF > 0 ? NF : N;
    int uu[kMaxN];
    const int16_t *ql = pl;
#pragma unroll
    for (int l = 0; l < kMaxN; ++l)
      if (l < NN) {
        uu[l] = *ql;
        ql += pstride;
      }
#pragma unroll
    for (int l = 0; l < kMaxN; ++l) {
      if (l < NN) {
        const double ud = (double)uu[l];
#pragma unroll
        for (int q = 0; q < L; ++q) acc[q] = fma(tab->wd[l][q], ud, acc[q]);
      }
    }
    uint32_t mag[L];
    const bool negative = crt_reduce<L>(acc, tab, mag);
    const int t = shift[i] + shift[lineB + j];
    chat = scaled_rn<L>(mag, t);
    if (negative) chat = -chat;
  }
  double out = __dmul_rn(alpha, chat);
  if (beta != 0.0) out = __dadd_rn(out, __dmul_rn(beta, C[i + j * ldc]));
  C[i + j * ldc] = out;
}

template <int L, int NF, bool GROUPED>
__global__ __launch_bounds__(256) void k_crt(Problem P1, Group G) {
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const int64_t nbx = (P.g.m + 255) / 256;
  const int64_t bx = local % nbx, j = local / nbx;
  crt_entry<L, NF>(P.w.planes, P.w.shift, P.w.flags, P.tab, P.g.N, P.g.m, P.g.mp, P.g.np,
               P.w.lineB, P.alpha, P.beta, P.C, P.ldc, bx * 256 + threadIdx.x, j);
}

__global__ void k_scal(int64_t m, double beta, double *__restrict__ C, int64_t ldc) {
  const int64_t nbx = (m + 255) / 256;
  const int64_t i = (int64_t)(blockIdx.x % nbx) * 256 + threadIdx.x;
  const int64_t j = blockIdx.x / nbx;
  if (i >= m) return;
  double *c = C + i + j * ldc;
  *c = beta == 0.0 ? 0.0 : __dmul_rn(beta, *c);
}

}  // namespace

hipError_t launch_crt_family(const Problem *P, const Group *G, int limbs, int N,
                             hipStream_t st) {
  const bool grouped = G != nullptr;
  Problem p1;
  Group g1;
  memset(&p1, 0, sizeof(p1));
  memset(&g1, 0, sizeof(g1));
  if (grouped)
    g1 = *G;
  else
    p1 = *P;
  const int64_t blocks = grouped ? G->total : family_blocks(kFamCrt, *P, 0);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), blk(256);
#define OZ2_CRT_LAUNCH(LL, NF)                                             \
  if (grouped)                                                             \
    hipLaunchKernelGGL((k_crt<LL, NF, true>), grid, blk, 0, st, p1, g1);   \
  else                                                                     \
    hipLaunchKernelGGL((k_crt<LL, NF, false>), grid, blk, 0, st, p1, g1);
  // the moduli counts of full accuracy (12-16) get kernels without
  // per-modulus branches
  if (limbs == 4 && N >= 12 && N <= 16) {
    switch (N) {
      case 12: OZ2_CRT_LAUNCH(4, 12) break;
      case 13: OZ2_CRT_LAUNCH(4, 13) break;
      case 14: OZ2_CRT_LAUNCH(4, 14) break;
      case 15: OZ2_CRT_LAUNCH(4, 15) break;
      default: OZ2_CRT_LAUNCH(4, 16) break;
    }
    return hipGetLastError();
  }
  if (limbs == 5 && N >= 14 && N <= 16) {
    switch (N) {
      case 14: OZ2_CRT_LAUNCH(5, 14) break;
      case 15: OZ2_CRT_LAUNCH(5, 15) break;
      default: OZ2_CRT_LAUNCH(5, 16) break;
    }
    return hipGetLastError();
  }
#define OZ2_CRT_CASE(LL)   \
  case LL:                 \
    OZ2_CRT_LAUNCH(LL, 0)  \
    break;
  switch (limbs) {
    OZ2_CRT_CASE(1)
    OZ2_CRT_CASE(2)
    OZ2_CRT_CASE(3)
    OZ2_CRT_CASE(4)
    OZ2_CRT_CASE(5)
    OZ2_CRT_CASE(6)
    OZ2_CRT_CASE(7)
    OZ2_CRT_CASE(8)
    OZ2_CRT_CASE(9)
    OZ2_CRT_CASE(10)
    default:
      return hipErrorInvalidValue;
  }
#undef OZ2_CRT_CASE
#undef OZ2_CRT_LAUNCH
  return hipGetLastError();
}

hipError_t launch_scal(int64_t m, int64_t n, double beta, double *C, int64_t ldc, hipStream_t st) {
  if (m == 0 || n == 0) return hipSuccess;
  const int64_t blocks = (m + 255) / 256 * n;
  if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scal, dim3((unsigned)blocks), dim3(256), 0, st, m, beta, C, ldc);
  return hipGetLastError();
}

}  // namespace oz2
