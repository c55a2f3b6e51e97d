// Scale exponents (Section III-E).
//
// Fast mode takes r_i from the Cauchy-Schwarz inequality instead: the squared
// norm of row i of Abar, summed exactly by the quantization pass; every line
// is then finalized from that exact value.  The accurate mode follows.
//
// For each row i of op(A) let r_i be the maximum over j of the bound product
// (Abar Bbar)_ij, and likewise c_j for the columns of op(B).  The scale
// exponent is e_i = max{e : 2^(2e+1) r_i <= P - 1}, giving log2 mu_i =
// log2 mu'_i + e_i; this makes 2 mu_i nu_j sum |a||b| < P (condition (3)),
// because each bound entry is at most sqrt(r_i c_j).
//
// The bound product runs on FP8 MFMA, so the computed maxima r'_i carry an
// error; the paper bounds it by (k - 1) 2^-24 (FP32 summation rounded to
// nearest), which gfx950's FP8 MFMA does not meet.  Each line is therefore
// decided from a window that holds the exact maximum under a stated worst
// case of the MFMA's accumulation (oz2_window.h).  When the whole window gives
// the same exponent, it is the exponent of the exact r_i.  Lines whose window
// straddles a threshold are recomputed exactly: Abar and Bbar are multiples
// of 2^-9 up to 256, so 2^18 (Abar Bbar)_ij is an integer below 2^52 for
// k <= 2^18 and is summed exactly in 64-bit integers.  The result is a
// deterministic function of the inputs, independent of the MFMA's summation
// order.  (Integer digit products stay exact: every product is an integer of
// magnitude <= 256, far inside the 2^-13 window, and every partial sum is at
// most 2^24.)
#include <string.h>

#include "oz2_device.h"
#include "oz2_internal.h"
#include "oz2_window.h"

namespace oz2 {

namespace {

template <bool GROUPED>
__global__ __launch_bounds__(256) void k_scale_decide(Problem P1, Group G) {
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const int64_t L = local * 256 + threadIdx.x;
  const int64_t lines = P.g.mp + P.g.np;
  if (L >= lines) return;
  const Work &w = P.w;
  const float r = __uint_as_float(w.rmax[L]);
  int ev = 0;
  if (r > 0.0f && !(w.flags[L] & kZeroLine)) {
    int e_small, e_large;
    window_exponents((double)r, P.g.kp, P.bparts, tables_of<GROUPED>(P1, G)->D, &e_small,
                     &e_large);
    ev = e_small;
    if (e_small != e_large) {
      // rows of op(A) from the front of the list, columns of op(B) from the back
      if (L < P.g.mp)
        w.amb[2 + atomicAdd(&w.amb[0], 1u)] = (uint32_t)L;
      else
        w.amb[1 + lines - atomicAdd(&w.amb[1], 1u)] = (uint32_t)L;
      w.flags[L] |= kFixup;
    }
  }
  w.e[L] = ev;
}

// Exact maxima of the bound product over the flagged lines.  With both
// factors multiples of 2^-9 up to 256, q9 = 2^9 x (an entry of Abar or Bbar)
// is an integer below 2^18 and every partial sum of q9 products is an integer
// below 2^52 (k <= 2^18), so FP64 fused multiply-adds sum them exactly, in any
// order.  The flagged lines of each side (rows of op(A), columns of op(B):
// the two ends of the list) are taken in groups of kFixG; an item is (group,
// chunk of kFixJ partner lines): the group's lines, decoded into LDS kFixKC k
// at a time, against one partner line per thread; the block's maximum per
// line goes to rfix (2^18 x the exact maximum) by an atomic maximum.  Each of
// the problem's nblk workgroups walks items blk, blk + nblk, ...
constexpr int kFixG = 2;   // few lines per item: many items, so many waves per SIMD
constexpr int kFixJ = 64;  // one wave per workgroup: small LDS, many workgroups per CU
constexpr int kFixKC = 256;

// One item with the group's first G lines (L[q] < 0: none): acc[q] = the exact
// bound product of line L[q] with partner line j (one per thread), k in
// chunks of kFixKC decoded into LDS; the partner's bytes of the next 64 k are
// loaded while the current 64 are summed.
template <int G>
__device__ __forceinline__ void fixup_item(const uint8_t *__restrict__ own_op, int64_t nown,
                                           int64_t base, const uint8_t *__restrict__ part,
                                           int64_t npart, int64_t kp, const int64_t (&L)[kFixG],
                                           int64_t j, double (*own)[kFixKC],
                                           const double *q9tab, uint64_t *__restrict__ rfix) {
  const int t = threadIdx.x;
  double acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) acc[q] = 0.0;
  const bool jv = j < npart;
  for (int64_t k0 = 0; k0 < kp; k0 += kFixKC) {  // kp is a multiple of kFixKC
    __syncthreads();  // the previous chunk's (or item's) readers are done
#pragma unroll
    for (int v = 0; v < G * kFixKC / kFixJ; ++v) {
      const int q = v / (kFixKC / kFixJ);
      const int h = (v % (kFixKC / kFixJ)) * kFixJ + t;
      double x = 0.0;
      if (L[q] >= 0) x = q9tab[own_op[kblocked(L[q] - base, k0 + h, nown)] & 0x7Fu];
      own[q][h] = x;
    }
    __syncthreads();
    if (jv) {
      // the partner's 64 bytes of each 64-k block are contiguous, blocks
      // 64 npart bytes apart
      const uint8_t *pj = part + kblocked(j, k0, npart);
      const int64_t step = npart * 64;
      constexpr int nb = kFixKC / 64;
      uint32_t cur[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) cur[w] = *(const uint32_t *)(pj + 4 * w);
      for (int b = 0; b < nb; ++b) {
        uint32_t nxt[16];
        if (b + 1 < nb) {
#pragma unroll
          for (int w = 0; w < 16; ++w) nxt[w] = *(const uint32_t *)(pj + (b + 1) * step + 4 * w);
        }
#pragma unroll 2
        for (int w = 0; w < 16; ++w) {
          const uint32_t word = cur[w];
#pragma unroll
          for (int z = 0; z < 4; ++z) {
            const double bv = q9tab[(word >> (8 * z)) & 0x7Fu];
            const int h = b * 64 + w * 4 + z;
#pragma unroll
            for (int q = 0; q < G; ++q) acc[q] = fma(own[q][h], bv, acc[q]);
          }
        }
        if (b + 1 < nb) {
#pragma unroll
          for (int w = 0; w < 16; ++w) cur[w] = nxt[w];
        }
      }
    }
  }
  // maxima per line over the wave's partners: exact integers below 2^52
#pragma unroll
  for (int q = 0; q < G; ++q) {
    if (L[q] < 0) continue;
    uint64_t m = jv ? (uint64_t)acc[q] : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(m, off, 64);
      m = o > m ? o : m;
    }
    if (t == 0 && m) atomicMax((unsigned long long *)&rfix[L[q]], (unsigned long long)m);
  }
}

__device__ __forceinline__ void scale_fixup(const uint8_t *__restrict__ Abar,
                                            const uint8_t *__restrict__ Bbar, int64_t mp,
                                            int64_t np, int64_t kp,
                                            const uint32_t *__restrict__ amb,
                                            uint64_t *__restrict__ rfix, int64_t blk,
                                            int64_t nblk) {
  __shared__ double own[kFixG][kFixKC];
  __shared__ double q9tab[128];
  const int t = threadIdx.x;
  for (int c = t; c < 128; c += kFixJ) q9tab[c] = (double)e4m3_q9((uint32_t)c);
  const int64_t lines = mp + np;
  const int64_t countA = amb[0], countB = amb[1];
  const int64_t groupsA = (countA + kFixG - 1) / kFixG, groupsB = (countB + kFixG - 1) / kFixG;
  // partners: the columns of op(B) for rows of op(A), and the other way
  const int64_t chunksA = (np + kFixJ - 1) / kFixJ, chunksB = (mp + kFixJ - 1) / kFixJ;
  const int64_t itemsA = groupsA * chunksA, items = itemsA + groupsB * chunksB;
  for (int64_t it = blk; it < items; it += nblk) {
    const int side = it < itemsA ? 0 : 1;  // 0: rows of op(A) against the columns of op(B)
    const int64_t r = side == 0 ? it : it - itemsA;
    const int64_t groups = side == 0 ? groupsA : groupsB;
    const int64_t g = r % groups, c = r / groups;
    const int64_t count = side == 0 ? countA : countB;
    const uint8_t *own_op = side == 0 ? Abar : Bbar;
    const uint8_t *part = side == 0 ? Bbar : Abar;
    const int64_t nown = side == 0 ? mp : np, npart = side == 0 ? np : mp;
    const int64_t base = side == 0 ? 0 : mp;  // line index of the side's first line
    // the group's lines (-1: none), the same in every thread; groups are
    // filled from the front, so the first n are valid
    int64_t L[kFixG];
#pragma unroll
    for (int q = 0; q < kFixG; ++q) {
      const int64_t e = g * kFixG + q;
      L[q] = e < count ? (int64_t)amb[side == 0 ? 2 + e : 1 + lines - e] : -1;
    }
    const int64_t n = count - g * kFixG;
    const int64_t j = c * kFixJ + t;
    if (n > 1)
      fixup_item<kFixG>(own_op, nown, base, part, npart, kp, L, j, own, q9tab, rfix);
    else
      fixup_item<1>(own_op, nown, base, part, npart, kp, L, j, own, q9tab, rfix);
  }
}

template <bool GROUPED>
__global__ __launch_bounds__(kFixJ) void k_scale_fixup(Problem P1, Group G) {
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Dims d = family_dims(kFamFixup, P);
  scale_fixup(P.w.Abar, P.w.Bbar, P.g.mp, P.g.np, P.g.kp, P.w.amb, P.w.rfix, local, d.x);
}

template <bool GROUPED>
__global__ __launch_bounds__(256) void k_scale_finalize(Problem P1, Group G) {
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const int64_t L = local * 256 + threadIdx.x;
  if (L >= P.g.mp + P.g.np) return;
  const Work &w = P.w;
  int ev = w.e[L];
  if (w.flags[L] & kFixup) {
    const uint64_t r18 = w.rfix[L];  // 2^18 x the exact line maximum, < 2^53
    ev = r18 ? exponent_rule(ldexp((double)r18, -18), tables_of<GROUPED>(P1, G)->D) : 0;
    w.e[L] = ev;
  }
  w.shift[L] = 7 - w.E[L] + ev;
}

}  // namespace

hipError_t launch_scale_family(int fam, const Problem *P, const Group *G, hipStream_t st) {
  const bool grouped = G != nullptr;
  Problem p1;
  Group g1;
  memset(&p1, 0, sizeof(p1));
  memset(&g1, 0, sizeof(g1));
  if (grouped)
    g1 = *G;
  else
    p1 = *P;
  const int64_t blocks = grouped ? G->total : family_blocks(fam, *P);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), blk(fam == kFamFixup ? kFixJ : 256);
#define OZ2_S(KER)                                             \
  if (grouped)                                                 \
    hipLaunchKernelGGL((KER<true>), grid, blk, 0, st, p1, g1); \
  else                                                         \
    hipLaunchKernelGGL((KER<false>), grid, blk, 0, st, p1, g1);
  switch (fam) {
    case kFamDecide: OZ2_S(k_scale_decide) break;
    case kFamFixup: OZ2_S(k_scale_fixup) break;
    case kFamFinal: OZ2_S(k_scale_finalize) break;
    default: return hipErrorInvalidValue;
  }
#undef OZ2_S
  return hipGetLastError();
}

}  // namespace oz2
