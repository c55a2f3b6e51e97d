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

#include "oz2_crt_math.h"
#include "oz2_internal.h"

namespace oz2 {

namespace {

// NF > 0: the number of moduli is the compile-time NF (no per-modulus
// branches); NF = 0: N at run time.
template <int L, int NF>
__device__ __forceinline__ void crt_entry(const int16_t *__restrict__ planes,
                                          const int32_t *__restrict__ shift,
                                          const uint32_t *__restrict__ flags,
                                          const Tables *__restrict__ tab, int N, int64_t m,
                                          int64_t mp, int64_t np, int64_t lineB, double alpha,
                                          double beta, double *__restrict__ C, int64_t ldc,
                                          int64_t i, int64_t j, int parts) {
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
    if (parts > 1) {
      // split-K: the residue products of each k part sit in their own copy
      // of the planes; their sum modulo p_l is the residue (|sum| < 2^12, so
      // the float quotient is within one and |u| <= p/2 + 1)
      const int64_t cstride = (int64_t)N * pstride;
#pragma unroll
      for (int l = 0; l < kMaxN; ++l)
        if (l < NN) {
          int sum = uu[l];
          for (int c = 1; c < parts; ++c) sum += pl[c * cstride + l * pstride];
          const int p = tab->p[l];
          uu[l] = sum - p * (int)rintf((float)sum * tab->inv_p[l]);
        }
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
  // block: 64 rows (one wave each) x 4 columns, so that outputs with few
  // rows leave few threads idle
  const int64_t nbx = (P.g.m + 63) / 64;
  const int64_t i = (local % nbx) * 64 + (threadIdx.x & 63);
  const int64_t j = (local / nbx) * 4 + (threadIdx.x >> 6);
  if (j >= P.g.n) return;
  crt_entry<L, NF>(P.w.planes, P.w.shift, P.w.flags, tables_of<GROUPED>(P1, G), P.g.N, P.g.m,
                   P.g.mp, P.g.np, P.w.lineB, P.alpha, P.beta, P.C, P.ldc, i, j, P.parts);
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
  const int64_t blocks = grouped ? G->total : family_blocks(kFamCrt, *P);
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
