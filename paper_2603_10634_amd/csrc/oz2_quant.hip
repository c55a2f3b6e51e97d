// Quantization passes over the FP64 inputs (HBM-bound):
//  - line maxima of op(A) rows / op(B) columns (for mu', nu', eq. def:mu'nu'),
//  - the round-up FP8 bound operands Abar, Bbar (Section III-E),
//  - the residues of A', B' for every modulus, split into FP8 digits
//    (eqs. def:A', def:B', CRTmatmul; digit splits of Sections III-B..III-D).
// Outputs are K-contiguous: line r's k values at r * kp, zero padded.
#include <string.h>

#include "oz2_device.h"
#include "oz2_internal.h"

namespace oz2 {

namespace {

constexpr uint64_t kAbsMask = 0x7FFFFFFFFFFFFFFFull;
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;

__device__ __forceinline__ void fill_zero(uint32_t *p, int64_t count, int64_t blk,
                                          int64_t nblk) {
  for (int64_t i = blk * 256 + threadIdx.x; i < count; i += nblk * 256) p[i] = 0u;
}

// Maxima of |x| over finite entries, per line; non-finite entries flag the line.
// Lines with contiguous k: one wave per line and k-chunk.
__device__ __forceinline__ void line_max_kcontig(const Operand &op, const LmaxShape &sh,
                                                 int64_t bx, int64_t by, uint64_t *amax,
                                                 uint32_t *flags) {
  const int lane = threadIdx.x & 63;
  const int64_t r = bx * 4 + (threadIdx.x >> 6);
  if (r >= op.lines) return;
  const int64_t h0 = by * sh.hchunk;
  const int64_t h1 = min(op.k, h0 + sh.hchunk);
  const double *row = op.ptr + r * op.sr;
  uint64_t m = 0;
  int bad = 0;
  for (int64_t h = h0 + lane; h < h1; h += 64) {
    uint64_t b = (uint64_t)__double_as_longlong(row[h]) & kAbsMask;
    if (b >= kInfBits)
      bad = 1;
    else
      m = b > m ? b : m;
  }
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  bad = __any(bad);
  if (lane == 0) {
    if (m) atomicMax((unsigned long long *)&amax[r], (unsigned long long)m);
    if (bad) atomicOr(&flags[r], kNonFinite);
  }
}

// Lines contiguous in memory: one thread per line, k split over blocks.
__device__ __forceinline__ void line_max_lcontig(const Operand &op, const LmaxShape &sh,
                                                 int64_t bx, int64_t by, uint64_t *amax,
                                                 uint32_t *flags) {
  const int64_t r = bx * 256 + threadIdx.x;
  if (r >= op.lines) return;
  const int64_t h0 = by * sh.hchunk;
  const int64_t h1 = min(op.k, h0 + sh.hchunk);
  uint64_t m = 0;
  int bad = 0;
  for (int64_t h = h0; h < h1; ++h) {
    uint64_t b = (uint64_t)__double_as_longlong(op.ptr[r + h * op.sh]) & kAbsMask;
    if (b >= kInfBits)
      bad = 1;
    else
      m = b > m ? b : m;
  }
  if (m) atomicMax((unsigned long long *)&amax[r], (unsigned long long)m);
  if (bad) atomicOr(&flags[r], kNonFinite);
}

template <bool GROUPED>
__global__ __launch_bounds__(256) void k_fill(Problem P1, Group G) {
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Dims d = family_dims(kFamFill, P, 0);
  fill_zero(P.w.zero, P.w.zero_words, local, d.x);
}

// SIDE 0: rows of op(A) (lines 0..mp-1), 1: columns of op(B) (lines mp..)
template <bool GROUPED, int SIDE>
__global__ __launch_bounds__(256) void k_line_max(Problem P1, Group G) {
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Operand &op = SIDE == 0 ? P.A : P.B;
  const int64_t base = SIDE == 0 ? 0 : P.g.mp;
  const LmaxShape sh = lmax_shape(op);
  const int64_t bx = local % sh.gx, by = local / sh.gx;
  if (op.sh == 1)
    line_max_kcontig(op, sh, bx, by, P.w.amax + base, P.w.flags + base);
  else
    line_max_lcontig(op, sh, bx, by, P.w.amax + base, P.w.flags + base);
}

constexpr int kTile = 64;        // lines x k per tile
constexpr int kTileLd = 65;      // LDS row stride (doubles)
static_assert(kTile == kQTile, "quantization tile");

// Stage a 64 x 64 tile of the operand (zero outside lines x k) in LDS as
// tile[line][h], loading along whichever dimension is contiguous.
template <bool LCONTIG>
__device__ __forceinline__ void load_tile(const double *__restrict__ x, int64_t lines, int64_t k,
                                          int64_t sr, int64_t sh, int64_t r0, int64_t h0,
                                          double *tile) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int a = idx >> 6, c = idx & 63;
    const int rr = LCONTIG ? c : a;
    const int hh = LCONTIG ? a : c;
    const int64_t r = r0 + rr, h = h0 + hh;
    double v = 0.0;
    if (r < lines && h < k) v = x[r * sr + h * sh];
    tile[rr * kTileLd + hh] = v;
  }
}

// FP8 round-up bound operand of one 64 x 64 tile (rows r0.., k h0..).
__device__ __forceinline__ void bound_operand_tile(const Operand &op, int64_t kp, int64_t r0,
                                                   int64_t h0, const uint64_t *amax, int32_t *E,
                                                   uint32_t *flags, uint8_t *bar, double *tile) {
  if (op.sr == 1)
    load_tile<true>(op.ptr, op.lines, op.k, op.sr, op.sh, r0, h0, tile);
  else
    load_tile<false>(op.ptr, op.lines, op.k, op.sr, op.sh, r0, h0, tile);
  __syncthreads();
  const int rl = threadIdx.x >> 2, b = threadIdx.x & 3;
  const int64_t r = r0 + rl;
  const uint64_t am = r < op.lines ? amax[r] : 0ull;
  const int Er = am ? ufp_exponent(am) : 0;
  if (h0 == 0 && b == 0) {
    E[r] = Er;
    if (am == 0) flags[r] |= kZeroLine;
  }
  const int sh7 = 7 - Er;  // mu' = 2^(7 - E)
  uint32_t packed[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t word = 0;
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const double v = tile[rl * kTileLd + b * 16 + w * 4 + z];
      const uint64_t bits = (uint64_t)__double_as_longlong(v);
      uint32_t code = 0;
      if ((bits & kAbsMask) < kInfBits) code = e4m3_round_up(bits, sh7);
      word |= code << (8 * z);
    }
    packed[w] = word;
  }
  uint4 out = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  *(uint4 *)(bar + r * kp + h0 + b * 16) = out;
}

template <bool GROUPED, int SIDE>
__global__ __launch_bounds__(256) void k_bound_operand(Problem P1, Group G) {
  __shared__ double tile[kTile * kTileLd];
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Operand &op = SIDE == 0 ? P.A : P.B;
  const int64_t base = SIDE == 0 ? 0 : P.g.mp;
  const Dims d = family_dims(SIDE == 0 ? kFamBarA : kFamBarB, P, 0);
  const int64_t bx = local % d.x, by = local / d.x;
  bound_operand_tile(op, P.g.kp, bx * kTile, by * kTile, P.w.amax + base, P.w.E + base,
                     P.w.flags + base, SIDE == 0 ? P.w.Abar : P.w.Bbar, tile);
}

// Residues of a' = sign * mf * 2^t (mf < 2^53 an integer held exactly in a
// double) modulo p, as an integer in [0, p).
__device__ __forceinline__ int residue_of(double mf, int t, const Tables *__restrict__ tab,
                                          int l, double pd, double inv) {
  double qd = floor(mf * inv);
  double rd = fma(-qd, pd, mf);  // exact: the result is an integer below 2p in magnitude
  if (rd < 0.0) rd += pd;
  if (rd >= pd) rd -= pd;
  int r = (int)rd;
  if (t > 0) {
    const int p = tab->p[l];
    int f;
    if (t < 256) {
      f = (tab->pow2hi[l][t >> 6] * tab->pow2lo[l][t & 63]) % p;
    } else {
      f = 1;
      for (int z = 0; z < t; ++z) f = (f * 2) % p;
    }
    r = (r * f) % p;
  }
  return r;
}

// Residues and FP8 digits of one 64 x 64 tile (rows r0.., k h0..).
__device__ __forceinline__ void residues_tile(const Operand &op, int64_t kp, int64_t lines_pad,
                                              int64_t r0, int64_t h0,
                                              const int32_t *__restrict__ shift,
                                              const Tables *__restrict__ tab, int N,
                                              uint8_t *__restrict__ slices, double *tile) {
  if (op.sr == 1)
    load_tile<true>(op.ptr, op.lines, op.k, op.sr, op.sh, r0, h0, tile);
  else
    load_tile<false>(op.ptr, op.lines, op.k, op.sr, op.sh, r0, h0, tile);
  __syncthreads();
  const int rl = threadIdx.x >> 2, b = threadIdx.x & 3;
  const int64_t r = r0 + rl;
  const int s = shift[r];  // log2(mu_r)

  // a' = trunc(a 2^s) = sign * mf * 2^t, exactly
  double mf[16];
  int tt[16];
  uint32_t neg = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const uint64_t bits = (uint64_t)__double_as_longlong(tile[rl * kTileLd + b * 16 + q]);
    mf[q] = 0.0;
    tt[q] = 0;
    if ((bits & kAbsMask) < kInfBits) {
      uint64_t mant;
      int qe;
      split_double(bits, mant, qe);
      const int e2 = qe + s;
      if (e2 >= 0) {
        mf[q] = (double)mant;
        tt[q] = e2;
      } else if (e2 > -64) {
        mf[q] = (double)(mant >> (-e2));
      }
      if (bits >> 63) neg |= 1u << q;
    }
  }

  const int64_t slice_stride = lines_pad * kp;
  uint8_t *base = slices + r * kp + h0 + b * 16;
  for (int l = 0; l < N; ++l) {
    const int p = tab->p[l];
    const int hlf = p >> 1;
    const int kind = tab->kind[l];
    const int srad = tab->s[l];
    const int smag = tab->smag[l];
    const double pd = (double)p, inv = tab->inv_pd[l];
    uint32_t w1[4] = {0, 0, 0, 0}, w2[4] = {0, 0, 0, 0}, w3[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      int u = residue_of(mf[q], tt[q], tab, l, pd, inv);
      if ((neg >> q) & 1u) u = -u;
      if (u > p - 1 - hlf) u -= p;  // symmetric range [-floor(p/2), ceil(p/2) - 1]
      if (u < -hlf) u += p;
      const int au = u < 0 ? -u : u;
      int x1, x2, x3 = 0;
      if (kind == 0) {
        // p = s^2: x1 = round(u / s) (ties away from zero), x2 = u - s x1
        int a1 = ((au + (srad >> 1)) * smag) >> 16;
        x1 = u < 0 ? -a1 : a1;
        x2 = u - srad * x1;
      } else {
        // s = 16: x1 = sign(u) ceil(|u| / 16), x2 = u - 16 x1, x3 = x1 + x2
        int a1 = (au + 15) >> 4;
        x1 = u < 0 ? -a1 : a1;
        x2 = u - 16 * x1;
        x3 = x1 + x2;
      }
      const int sh8 = 8 * (q & 3);
      w1[q >> 2] |= e4m3_of_small_int(x1) << sh8;
      w2[q >> 2] |= e4m3_of_small_int(x2) << sh8;
      w3[q >> 2] |= e4m3_of_small_int(x3) << sh8;
    }
    uint8_t *dst = base + (int64_t)tab->slice0[l] * slice_stride;
    *(uint4 *)dst = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    *(uint4 *)(dst + slice_stride) = make_uint4(w2[0], w2[1], w2[2], w2[3]);
    if (kind != 0) *(uint4 *)(dst + 2 * slice_stride) = make_uint4(w3[0], w3[1], w3[2], w3[3]);
  }
}

template <bool GROUPED, int SIDE>
__global__ __launch_bounds__(256) void k_residues(Problem P1, Group G) {
  __shared__ double tile[kTile * kTileLd];
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Operand &op = SIDE == 0 ? P.A : P.B;
  const int64_t base = SIDE == 0 ? 0 : P.g.mp;
  const Dims d = family_dims(SIDE == 0 ? kFamResA : kFamResB, P, 0);
  const int64_t bx = local % d.x, by = local / d.x;
  residues_tile(op, P.g.kp, SIDE == 0 ? P.g.mp : P.g.np, bx * kTile, by * kTile,
                P.w.shift + base, P.tab, P.g.N, SIDE == 0 ? P.w.Asl : P.w.Bsl, tile);
}

}  // namespace

hipError_t launch_quant_family(int fam, const Problem *P, const Group *G, hipStream_t st) {
  const bool grouped = G != nullptr;
  Problem p1;
  Group g1;
  memset(&p1, 0, sizeof(p1));
  memset(&g1, 0, sizeof(g1));
  if (grouped)
    g1 = *G;
  else
    p1 = *P;
  const int64_t blocks = grouped ? G->total : family_blocks(fam, *P, 0);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), blk(256);
#define OZ2_Q(KER)                                                          \
  if (grouped)                                                              \
    hipLaunchKernelGGL((KER<true>), grid, blk, 0, st, p1, g1);              \
  else                                                                      \
    hipLaunchKernelGGL((KER<false>), grid, blk, 0, st, p1, g1);
#define OZ2_Q2(KER, SIDE)                                                   \
  if (grouped)                                                              \
    hipLaunchKernelGGL((KER<true, SIDE>), grid, blk, 0, st, p1, g1);        \
  else                                                                      \
    hipLaunchKernelGGL((KER<false, SIDE>), grid, blk, 0, st, p1, g1);
  switch (fam) {
    case kFamFill: OZ2_Q(k_fill) break;
    case kFamLmaxA: OZ2_Q2(k_line_max, 0) break;
    case kFamLmaxB: OZ2_Q2(k_line_max, 1) break;
    case kFamBarA: OZ2_Q2(k_bound_operand, 0) break;
    case kFamBarB: OZ2_Q2(k_bound_operand, 1) break;
    case kFamResA: OZ2_Q2(k_residues, 0) break;
    case kFamResB: OZ2_Q2(k_residues, 1) break;
    default: return hipErrorInvalidValue;
  }
#undef OZ2_Q
#undef OZ2_Q2
  return hipGetLastError();
}

}  // namespace oz2
