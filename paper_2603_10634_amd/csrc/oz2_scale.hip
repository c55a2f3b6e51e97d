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
    window_exponents((double)r, P.g.kp, P.bparts, P.tab->D, &e_small, &e_large);
    ev = e_small;
    if (e_small != e_large) {
      const uint32_t slot = atomicAdd(&w.amb[0], 1u);
      w.amb[1 + slot] = (uint32_t)L;
      w.flags[L] |= kFixup;
    }
  }
  w.e[L] = ev;
}

// Exact maxima of the bound product over the flagged lines.  With both
// factors multiples of 2^-9 up to 256, q9 = 2^9 x (an entry of Abar or Bbar)
// is an integer below 2^18 and every partial sum of q9 products is an integer
// below 2^52 (k <= 2^18), so FP64 fused multiply-adds sum them exactly, in any
// order.  The flagged lines are taken in groups of kFixG consecutive list
// entries; an item is (side, group, chunk of kFixJ partner lines): the group's
// lines of that side (rows of op(A), or columns of op(B)), decoded into LDS
// kFixKC k at a time, against one partner line per thread; the block's
// maximum per line goes to rfix (2^18 x the exact maximum) by an atomic
// maximum.  Each of the problem's nblk workgroups walks items blk, blk + nblk..
constexpr int kFixG = 8;
constexpr int kFixKC = 512;
constexpr int kFixJ = 256;

__device__ __forceinline__ void scale_fixup(const uint8_t *__restrict__ Abar,
                                            const uint8_t *__restrict__ Bbar, int64_t mp,
                                            int64_t np, int64_t kp,
                                            const uint32_t *__restrict__ amb,
                                            uint64_t *__restrict__ rfix, int64_t blk,
                                            int64_t nblk) {
  __shared__ double own[kFixG][kFixKC];
  __shared__ double q9tab[128];
  const int t = threadIdx.x;
  if (t < 128) q9tab[t] = (double)e4m3_q9((uint32_t)t);
  const int64_t count = amb[0];
  const int64_t groups = (count + kFixG - 1) / kFixG;
  const int64_t chunks = ((mp > np ? mp : np) + kFixJ - 1) / kFixJ;
  const int64_t items = 2 * groups * chunks;
  for (int64_t it = blk; it < items; it += nblk) {
    const int side = (int)(it & 1);  // 0: rows of op(A) against the columns of op(B)
    const int64_t g = (it >> 1) % groups, c = (it >> 1) / groups;
    const uint8_t *own_op = side == 0 ? Abar : Bbar;
    const uint8_t *part = side == 0 ? Bbar : Abar;
    const int64_t nown = side == 0 ? mp : np, npart = side == 0 ? np : mp;
    const int64_t base = side == 0 ? 0 : mp;  // line index of the side's first line
    // the group's lines of this side (-1: none), the same in every thread
    int64_t L[kFixG];
    bool any = false;
#pragma unroll
    for (int q = 0; q < kFixG; ++q) {
      const int64_t e = g * kFixG + q;
      const int64_t l = e < count ? (int64_t)amb[1 + e] : -1;
      L[q] = l >= 0 && (l < mp) == (side == 0) ? l : -1;
      any |= L[q] >= 0;
    }
    if (!any || c * kFixJ >= npart) continue;
    const int64_t j = c * kFixJ + t;
    double acc[kFixG];
#pragma unroll
    for (int q = 0; q < kFixG; ++q) acc[q] = 0.0;
    for (int64_t k0 = 0; k0 < kp; k0 += kFixKC) {
      const int kc = kp - k0 < kFixKC ? (int)(kp - k0) : kFixKC;  // 256 or 512
      __syncthreads();  // the previous chunk's (or item's) readers are done
#pragma unroll
      for (int v = 0; v < kFixG * kFixKC / kFixJ; ++v) {
        const int q = v / (kFixKC / kFixJ);
        const int h = (v % (kFixKC / kFixJ)) * kFixJ + t;
        double x = 0.0;
        if (L[q] >= 0 && h < kc)
          x = q9tab[own_op[kblocked(L[q] - base, k0 + h, nown)] & 0x7Fu];
        own[q][h] = x;
      }
      __syncthreads();
      if (j < npart) {
        for (int h = 0; h < kc; h += 8) {
          // 8 bytes at h (h % 8 == 0) sit in one 64-byte piece of the line
          const uint64_t b8 = *(const uint64_t *)(part + kblocked(j, k0 + h, npart));
#pragma unroll
          for (int z = 0; z < 8; ++z) {
            const double b = q9tab[(uint32_t)(b8 >> (8 * z)) & 0x7Fu];
#pragma unroll
            for (int q = 0; q < kFixG; ++q) acc[q] = fma(own[q][h + z], b, acc[q]);
          }
        }
      }
    }
    // block maxima per line: exact integers below 2^52
#pragma unroll
    for (int q = 0; q < kFixG; ++q) {
      if (L[q] < 0) continue;
      uint64_t m = (uint64_t)acc[q];
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
      }
      if ((t & 63) == 0 && m) atomicMax((unsigned long long *)&rfix[L[q]], (unsigned long long)m);
    }
  }
}

template <bool GROUPED>
__global__ __launch_bounds__(256) void k_scale_fixup(Problem P1, Group G) {
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
    ev = r18 ? exponent_rule(ldexp((double)r18, -18), P.tab->D) : 0;
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
  const dim3 grid((unsigned)blocks), blk(256);
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
