// Chinese-remainder reconstruction and inverse scaling (eqs.
// CRT_finalreduction, inversescaling), fused with alpha/beta.
//
// Per output entry (i, j): u_l = C'_l mod p_l in [0, p_l) from the int16
// planes; S = sum_l w_l u_l + floor(P/2) in 32-bit limbs (exact); R = S mod P;
// C' = R - floor(P/2), which lies in (-P/2, P/2) by condition (3).  Then
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
    // S = sum_l w_l u_l + floor(P/2), accumulated per 32-bit limb in FP64
    // (full rate on this GPU, unlike 64-bit integer multiply-adds): every
    // limb sum stays below 2^32 (1 + 33 * 1089) < 2^48, so it is exact
    double acc[L];
#pragma unroll
    for (int q = 0; q < L; ++q) acc[q] = (double)tab->half[q];
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
        const int u = uu[l] + (tab->p[l] & (uu[l] >> 31));  // C'_l mod p_l in [0, p_l)
        const double ud = (double)u;
#pragma unroll
        for (int q = 0; q < L; ++q) acc[q] = fma(tab->wd[l][q], ud, acc[q]);
      }
    }
    // carry-propagate into 32-bit limbs: t = acc + carry < 2^49, split exactly
    uint32_t S[L + 1];
    double carry = 0.0;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const double t = acc[q] + carry;
      const double hi = floor(t * 0x1p-32);
      S[q] = (uint32_t)fma(-hi, 0x1p32, t);
      carry = hi;
    }
    S[L] = (uint32_t)carry;
    // quotient estimate t ~ S / P (S < 2^16 P), then R = S - t P, corrected once
    double sd = 0.0;
#pragma unroll
    for (int q = 0; q <= L; ++q) sd += ldexp((double)S[q], 32 * q);
    int64_t tq = (int64_t)floor(sd * tab->inv_P_d);
    if (tq < 0) tq = 0;
    uint32_t R[L + 1];
    int64_t borrow = 0;
    uint64_t mulc = 0;
#pragma unroll
    for (int q = 0; q <= L; ++q) {
      const uint64_t pq = (q < L) ? (uint64_t)tab->P[q] : 0ull;
      const uint64_t prod = pq * (uint64_t)tq + mulc;
      mulc = prod >> 32;
      const int64_t d = (int64_t)S[q] - (int64_t)(uint32_t)prod + borrow;
      R[q] = (uint32_t)d;
      borrow = d >> 32;  // 0 or -1
    }
    // R is now S - tq P as a two's-complement (L+1)-limb number
    const bool negR = (R[L] >> 31) != 0;
    if (negR) {  // add P back
      uint64_t c = 0;
#pragma unroll
      for (int q = 0; q <= L; ++q) {
        const uint64_t t = (uint64_t)R[q] + ((q < L) ? tab->P[q] : 0u) + c;
        R[q] = (uint32_t)t;
        c = t >> 32;
      }
    } else {  // subtract P if R >= P
      bool ge = R[L] != 0;
      bool decided = ge;
#pragma unroll
      for (int q = L - 1; q >= 0; --q) {
        if (!decided && R[q] != tab->P[q]) {
          ge = R[q] > tab->P[q];
          decided = true;
        }
      }
      if (!decided) ge = true;  // equal
      if (ge) {
        int64_t b = 0;
#pragma unroll
        for (int q = 0; q <= L; ++q) {
          const int64_t d = (int64_t)R[q] - (int64_t)((q < L) ? tab->P[q] : 0u) + b;
          R[q] = (uint32_t)d;
          b = d >> 32;
        }
      }
    }
    // C' = R - floor(P/2): magnitude and sign
    bool ge = false, decided = false;
#pragma unroll
    for (int q = L - 1; q >= 0; --q) {
      if (!decided && R[q] != tab->half[q]) {
        ge = R[q] > tab->half[q];
        decided = true;
      }
    }
    if (!decided) ge = true;
    uint32_t mag[L];
    int64_t b = 0;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const int64_t d = ge ? (int64_t)R[q] - (int64_t)tab->half[q] + b
                           : (int64_t)tab->half[q] - (int64_t)R[q] + b;
      mag[q] = (uint32_t)d;
      b = d >> 32;
    }
    const int t = shift[i] + shift[lineB + j];
    chat = scaled_rn<L>(mag, t);
    if (!ge) chat = -chat;
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
