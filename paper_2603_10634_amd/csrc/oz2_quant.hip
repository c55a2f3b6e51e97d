// Quantization passes over the FP64 inputs (HBM-bound):
//  - line maxima of op(A) rows / op(B) columns (for mu', nu', eq. def:mu'nu'),
//  - the round-up FP8 bound operands Abar, Bbar (Section III-E), or in fast
//    mode the squared norms of their lines (Cauchy-Schwarz bound),
//  - the residues of A', B' for every modulus, split into FP8 digits
//    (eqs. def:A', def:B', CRTmatmul; digit splits of Sections III-B..III-D).
// Outputs are k-blocked (kblocked in oz2_internal.h), zero padded.
#include <string.h>

#include "oz2_device.h"
#include "oz2_internal.h"

namespace oz2 {

namespace {

constexpr uint64_t kAbsMask = 0x7FFFFFFFFFFFFFFFull;
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;
// class mask of the finite nonzero doubles (negative and positive normal and
// subnormal numbers)
constexpr int kFiniteNonzero = 0x198;

__device__ __forceinline__ void fill_zero(uint32_t *p, int64_t count, int64_t blk,
                                          int64_t nblk) {
  for (int64_t i = blk * 256 + threadIdx.x; i < count; i += nblk * 256) p[i] = 0u;
}

constexpr int kLmaxU = 8;  // independent loads per trip of the line-maximum loops

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
  int64_t h = h0 + lane;
  // kLmaxU loads in flight per trip, then a remainder of single loads
  for (; h + 64 * (kLmaxU - 1) < h1; h += 64 * kLmaxU) {
    uint64_t b[kLmaxU];
#pragma unroll
    for (int u = 0; u < kLmaxU; ++u)
      b[u] = (uint64_t)__double_as_longlong(row[h + 64 * u]) & kAbsMask;
#pragma unroll
    for (int u = 0; u < kLmaxU; ++u) {
      if (b[u] >= kInfBits)
        bad = 1;
      else
        m = b[u] > m ? b[u] : m;
    }
  }
  for (; h < h1; h += 64) {
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
  int64_t h = h0;
  for (; h + kLmaxU <= h1; h += kLmaxU) {
    uint64_t b[kLmaxU];
#pragma unroll
    for (int u = 0; u < kLmaxU; ++u)
      b[u] = (uint64_t)__double_as_longlong(op.ptr[r + (h + u) * op.sh]) & kAbsMask;
#pragma unroll
    for (int u = 0; u < kLmaxU; ++u) {
      if (b[u] >= kInfBits)
        bad = 1;
      else
        m = b[u] > m ? b[u] : m;
    }
  }
  for (; h < h1; ++h) {
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
  const Dims d = family_dims(kFamFill, P);
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

// Quantization tiles: 16 lines x 128 k per workgroup of 256 threads; thread t
// owns line t / 16 and the 8 consecutive k (t % 16) * 8 .. + 7, so a line's
// bytes of a tile leave as one 128-byte segment per output slice.  Small
// tiles and 8 inputs per thread keep the register and LDS footprint low, so
// many waves stream through each CU.  The FP64
// tile is staged in LDS to read along whichever dimension is contiguous;
// element h of a row sits at h + h / 16 (one pad double per 16) so that the
// threads of one read (same q, consecutive t) fall into different banks.
constexpr int kRowLd = kQK + kQK / 16 + 1;   // 137 doubles per staged row

__device__ __forceinline__ int tile_at(int rr, int hh) { return rr * kRowLd + hh + (hh >> 4); }

template <bool LCONTIG, int QL>
__device__ __forceinline__ void load_tile(const double *__restrict__ x, int64_t lines, int64_t k,
                                          int64_t sr, int64_t sh, int64_t r0, int64_t h0,
                                          double *tile) {
#pragma unroll
  for (int q = 0; q < QL * kQK / 256; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int rr = LCONTIG ? (idx % QL) : (idx >> 7);
    const int hh = LCONTIG ? (idx / QL) : (idx & 127);
    const int64_t r = r0 + rr, h = h0 + hh;
    double v = 0.0;
    if (r < lines && h < k) v = x[r * sr + h * sh];
    tile[tile_at(rr, hh)] = v;
  }
}

template <int QL = kQL>
__device__ __forceinline__ void stage_tile(const Operand &op, int64_t r0, int64_t h0,
                                           double *tile) {
  if (op.sr == 1)
    load_tile<true, QL>(op.ptr, op.lines, op.k, op.sr, op.sh, r0, h0, tile);
  else
    load_tile<false, QL>(op.ptr, op.lines, op.k, op.sr, op.sh, r0, h0, tile);
}

// FP8 round-up bound operand of one tile (lines r0.., k h0..).
__device__ __forceinline__ void bound_operand_tile(const Operand &op, int64_t lines_pad,
                                                   int64_t r0, int64_t h0, const uint64_t *amax,
                                                   int32_t *E, uint32_t *flags, uint8_t *bar,
                                                   double *tile) {
  stage_tile(op, r0, h0, tile);
  __syncthreads();
  const int rl = threadIdx.x >> 4, b = threadIdx.x & 15;
  const int64_t r = r0 + rl;
  const uint64_t am = r < op.lines ? amax[r] : 0ull;
  const int Er = am ? ufp_exponent(am) : 0;
  if (h0 == 0 && b == 0) {
    E[r] = Er;
    if (am == 0) flags[r] |= kZeroLine;
  }
  const int sh7 = 7 - Er;  // mu' = 2^(7 - E)
  uint32_t packed[2];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    uint32_t word = 0;
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const double v = tile[tile_at(rl, b * 8 + w * 4 + z)];
      const uint32_t code =
          __builtin_amdgcn_class(v, kFiniteNonzero) ? e4m3_round_up(v, sh7) : 0u;
      word |= code << (8 * z);
    }
    packed[w] = word;
  }
  *(uint2 *)(bar + kblocked(r, h0 + b * 8, lines_pad)) = make_uint2(packed[0], packed[1]);
}

template <bool GROUPED, int SIDE>
__global__ __launch_bounds__(256) void k_bound_operand(Problem P1, Group G) {
  __shared__ double tile[kQL * kRowLd];
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Operand &op = SIDE == 0 ? P.A : P.B;
  const int64_t base = SIDE == 0 ? 0 : P.g.mp;
  const Dims d = family_dims(SIDE == 0 ? kFamBarA : kFamBarB, P);
  const int64_t bx = local % d.x, by = local / d.x;
  bound_operand_tile(op, SIDE == 0 ? P.g.mp : P.g.np, bx * kQL, by * kQK, P.w.amax + base,
                     P.w.E + base, P.w.flags + base, SIDE == 0 ? P.w.Abar : P.w.Bbar, tile);
}

// Fast mode: 2^18 x the squared Euclidean norm of every line of the round-up
// bound operand over one tile, added to norm[r] (Section III-E, the
// Cauchy-Schwarz bound; with r_i, c_j these norms, the bound product obeys
// (Abar Bbar)_ij <= sqrt(r_i c_j)).  Abar is not stored.  Each 2^9 Abar is an
// integer of at most 2^17, so the sums are exact 64-bit integers (at most
// 2^52 for k <= 2^18) and do not depend on the order of the additions.
// Every line is flagged to take its exponent from this exact value.
__device__ __forceinline__ void bound_norm_tile(const Operand &op, int64_t r0, int64_t h0,
                                                const uint64_t *amax, int32_t *E,
                                                uint32_t *flags, uint64_t *norm,
                                                double *tile) {
  stage_tile(op, r0, h0, tile);
  __syncthreads();
  const int rl = threadIdx.x >> 4, b = threadIdx.x & 15;
  const int64_t r = r0 + rl;
  const uint64_t am = r < op.lines ? amax[r] : 0ull;
  const int Er = am ? ufp_exponent(am) : 0;
  if (h0 == 0 && b == 0) {
    E[r] = Er;
    flags[r] |= am ? kFixup : (kFixup | kZeroLine);
  }
  const int sh7 = 7 - Er;  // mu' = 2^(7 - E)
  uint64_t sum = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double v = tile[tile_at(rl, b * 8 + q)];
    const uint32_t q9 =
        __builtin_amdgcn_class(v, kFiniteNonzero) ? e4m3_q9(e4m3_round_up(v, sh7)) : 0u;
    sum += (uint64_t)q9 * q9;
  }
  // the 16 threads of a line are 16 consecutive lanes
  sum += __shfl_xor(sum, 1, 64);
  sum += __shfl_xor(sum, 2, 64);
  sum += __shfl_xor(sum, 4, 64);
  sum += __shfl_xor(sum, 8, 64);
  if (b == 0 && sum) atomicAdd((unsigned long long *)&norm[r], (unsigned long long)sum);
}

template <bool GROUPED, int SIDE>
__global__ __launch_bounds__(256) void k_bound_norm(Problem P1, Group G) {
  __shared__ double tile[kQL * kRowLd];
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Operand &op = SIDE == 0 ? P.A : P.B;
  const int64_t base = SIDE == 0 ? 0 : P.g.mp;
  const Dims d = family_dims(SIDE == 0 ? kFamNormA : kFamNormB, P);
  const int64_t bx = local % d.x, by = local / d.x;
  bound_norm_tile(op, bx * kQL, by * kQK, P.w.amax + base, P.w.E + base, P.w.flags + base,
                  P.w.rfix + base, tile);
}

// Residues of a' (eq. def:A') for every modulus, split into digits, for one
// tile (lines r0.., k h0..).
//
// Each finite nonzero input is |a| = F 2^(E - 53) with E its frexp exponent
// and F < 2^53 an integer (also for subnormal a); with s = log2 mu_r the
// integer is a' = sign (F 2^t) for t = E - 53 + s > 0, else sign floor(F 2^t)
// (eq. def:A': truncation toward zero).  Per input the signed integer
// x = sign F 2^min(t, 10) (t > 0) or a' (t <= 0) is held exactly in a double
// (|x| < 2^63): x = trunc(a 2^(s - max(t - 10, 0))), where the scaling is
// exact whenever the result is at least 2^-1022 and otherwise is below one in
// magnitude, so that the truncation gives zero either way.  Zero, infinite and
// NaN inputs give x = +0 (their lines are flagged, or their digits are zero).
// One FP64 step serves two consecutive moduli p, p' of one kind (R = p p' <
// 2^21), or one modulus alone (R = p): q = rint(x R^-1) is within
// 2^63 / R 2^-52 = 2^11 / R of x / R (both roundings), so
// |f| = |x - q R| < R / 2 + 2^11 < 2^20 + 2^11, and f is exact in one fused
// multiply-add.  Per modulus, one FP32 step f - p rint(f p^-1) then removes
// the nearest multiple of p: the computed quotient is within
// |f / p| 2^-23 < 1 / (8p) (1 + 2^-9) of f / p (f is exact in FP32), while
// for odd p an integer f / p is at least 1 / (2p) from a tie,
// so the result is exactly in [-(p - 1)/2, (p - 1)/2]; for even p it is
// in [-p/2, p/2] and a tie's +p/2 is moved to -p/2, giving the symmetric
// range [-floor(p/2), ceil(p/2) - 1] in both cases.  Inputs with t > 10 (only
// for large N: t <= e - 45 for the scale exponent e) are multiplied by
// 2^(t - 10) mod p (tables) and reduced by the same FP32 step (products below
// p^2 / 2 < 2^20, exact; quotient error below p 2^-24 < 1 / (2p) for
// p < 2896).  Digits (Sections
// III-B, III-C) are formed in FP32, exact for these small integers, and
// packed to E4M3 two at a time by the hardware conversion (exact: every digit
// has |d| <= 16).  An INT8 modulus (Section II) stores the residue itself,
// in [-128, 127], as one INT8 byte.  The moduli are visited kind by kind
// (squares, then Karatsuba, then INT8), so no loop body branches on the kind.
constexpr int kDirectT = 10;  // powers 2^t applied in FP64 directly

constexpr int kRE = kQK * kQL / 256;  // inputs per thread of a quantization tile (8)

struct ResidueIn {
  double x[kRE];  // sign F 2^min(t, 10) (t > 0) or signed a' (t <= 0), exact, never -0
  int t[kRE];     // t > 10: the power of two t - 10 still to apply, else 0
};

// HUGE: some lane of the wave has t > 10 (a wave-uniform choice of the
// whole modulus loop, so that the common loop carries nothing of the table
// lookup of 2^(t - 10) mod p).
// The FP64 step: f = x - R rint(x R^-1), exact, |f| < 2^20 + 2^11.
__device__ __forceinline__ void fp64_step(const ResidueIn &in, double R, double invR,
                                          float (&f)[kRE]) {
#pragma unroll
  for (int q = 0; q < kRE; ++q) f[q] = (float)fma(-rint(in.x[q] * invR), R, in.x[q]);
}

template <int KIND, bool EVEN, bool HUGE>
__device__ __forceinline__ void modulus_pass(const float (&f)[kRE], const ResidueIn &in,
                                             const Tables *__restrict__ tab, int l, uint8_t *dst,
                                             int64_t slice_stride) {
  const int p = tab->p[l];
  const float pf = (float)p;
  const float hif = (float)(p - 1 - (p >> 1));
  const float invpf = tab->inv_p[l];
  float fu[kRE];
#pragma unroll
  for (int q = 0; q < kRE; ++q) fu[q] = fmaf(-rintf(f[q] * invpf), pf, f[q]);
  if (HUGE) {
#pragma unroll
    for (int q = 0; q < kRE; ++q) {
      if (in.t[q] > 0) {
        const float prod = fu[q] * (float)tab->pw[l][in.t[q]];
        fu[q] = fmaf(-rintf(prod * invpf), pf, prod);
      }
    }
  }
  if (EVEN) {
    // a tie leaves +p/2, which belongs to -p/2
#pragma unroll
    for (int q = 0; q < kRE; ++q) fu[q] = fu[q] > hif ? fu[q] - pf : fu[q];
  }
  constexpr int G = kRE / 4;
  int w1[G], w2[G], w3[G];
  if (KIND == 2) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      uint32_t word = 0;
#pragma unroll
      for (int z = 0; z < 4; ++z) word |= ((uint32_t)(int)fu[4 * g + z] & 0xFFu) << (8 * z);
      w1[g] = (int)word;
    }
    *(uint2 *)dst = make_uint2(w1[0], w1[1]);
    return;
  }
  const float sf = (float)tab->s[l], invs = tab->inv_s[l];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    float x1[4], x2[4], x3[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const float f = fu[4 * g + z];
      if (KIND == 0) {
        // p = s^2: x1 = round(u / s) (ties away from zero), x2 = u - s x1;
        // for odd s, u / s is never a tie and rint rounds to the nearest
        const float tq = f * invs;
        if (EVEN)
          x1[z] = truncf(tq + copysignf(0.5f, tq)) + 0.0f;  // + 0 turns -0 into +0
        else
          x1[z] = rintf(tq) + 0.0f;
        x2[z] = fmaf(-sf, x1[z], f);
      } else {
        // s = 16: x1 = sign(u) ceil(|u| / 16), x2 = u - 16 x1, x3 = x1 + x2
        x1[z] = copysignf(ceilf(fabsf(f) * 0.0625f), f);
        x2[z] = fmaf(-16.0f, x1[z], f);
        x3[z] = x1[z] + x2[z];
      }
    }
    // the first conversion's old word is a register no longer needed (the
    // residues themselves): its upper half is replaced by the second one
    w1[g] = __builtin_amdgcn_cvt_pk_fp8_f32(x1[0], x1[1], __float_as_int(fu[4 * g]), false);
    w1[g] = __builtin_amdgcn_cvt_pk_fp8_f32(x1[2], x1[3], w1[g], true);
    w2[g] = __builtin_amdgcn_cvt_pk_fp8_f32(x2[0], x2[1], __float_as_int(fu[4 * g + 1]), false);
    w2[g] = __builtin_amdgcn_cvt_pk_fp8_f32(x2[2], x2[3], w2[g], true);
    if (KIND == 1) {
      w3[g] = __builtin_amdgcn_cvt_pk_fp8_f32(x3[0], x3[1], __float_as_int(fu[4 * g + 2]), false);
      w3[g] = __builtin_amdgcn_cvt_pk_fp8_f32(x3[2], x3[3], w3[g], true);
    }
  }
  *(uint2 *)dst = make_uint2(w1[0], w1[1]);
  *(uint2 *)(dst + slice_stride) = make_uint2(w2[0], w2[1]);
  if (KIND == 1) *(uint2 *)(dst + 2 * slice_stride) = make_uint2(w3[0], w3[1]);
}

template <int KIND, bool HUGE>
__device__ __forceinline__ void one_modulus(const float (&f)[kRE], const ResidueIn &in,
                                            const Tables *__restrict__ tab, int l, uint8_t *base,
                                            int64_t slice_stride) {
  uint8_t *dst = base + (int64_t)tab->slice0[l] * slice_stride;
  // p is uniform: the parity test is a branch, not a select
  if (tab->p[l] & 1)
    modulus_pass<KIND, false, HUGE>(f, in, tab, l, dst, slice_stride);
  else
    modulus_pass<KIND, true, HUGE>(f, in, tab, l, dst, slice_stride);
}

// The moduli l0 .. l1 - 1 of one kind, two per FP64 step (one per step on
// the rare path with t > 10, which holds more registers).
template <int KIND, bool HUGE>
__device__ __forceinline__ void kind_moduli(const ResidueIn &in, const Tables *__restrict__ tab,
                                            int l0, int l1, uint8_t *base, int64_t slice_stride) {
  int l = l0;
  for (; !HUGE && l + 1 < l1; l += 2) {
    float f[kRE];
    fp64_step(in, (double)(tab->p[l] * tab->p[l + 1]), tab->inv_pair[l], f);
    one_modulus<KIND, HUGE>(f, in, tab, l, base, slice_stride);
    one_modulus<KIND, HUGE>(f, in, tab, l + 1, base, slice_stride);
  }
  for (; l < l1; ++l) {
    float f[kRE];
    fp64_step(in, (double)tab->p[l], tab->inv_pd[l], f);
    one_modulus<KIND, HUGE>(f, in, tab, l, base, slice_stride);
  }
}

// Every modulus of one thread's inputs, kind by kind.
template <bool HUGE>
__device__ __forceinline__ void residue_moduli(const ResidueIn &in, const Tables *__restrict__ tab,
                                               int N, int nsq, int nka, uint8_t *base,
                                               int64_t slice_stride) {
  kind_moduli<0, HUGE>(in, tab, 0, nsq, base, slice_stride);
  kind_moduli<1, HUGE>(in, tab, nsq, nsq + nka, base, slice_stride);
  kind_moduli<2, HUGE>(in, tab, nsq + nka, N, base, slice_stride);
}

__device__ __forceinline__ void residues_tile(const Operand &op, int64_t kp, int64_t lines_pad,
                                              int64_t r0, int64_t h0,
                                              const int32_t *__restrict__ shift,
                                              const Tables *__restrict__ tab, int N, int nsq,
                                              int nka, uint8_t *__restrict__ slices,
                                              double *tile) {
  stage_tile(op, r0, h0, tile);
  __syncthreads();
  // thread t: line t / 16, the kRE = 8 consecutive k (t % 16) * 8 .. + 7
  const int rl = threadIdx.x >> 4, b = threadIdx.x & 15;
  const int64_t r = r0 + rl;
  const int s = shift[r];  // log2(mu_r)

  ResidueIn in;
  bool huge = false;
#pragma unroll
  for (int q = 0; q < kRE; ++q) {
    const double a = tile[tile_at(rl, b * kRE + q)];
    const bool nz = __builtin_amdgcn_class(a, kFiniteNonzero);
    int t = nz ? __builtin_amdgcn_frexp_exp(a) - 53 + s : 0;
    t = t < kPowT ? t : kPowT - 1;
    const int tt = t > kDirectT ? t - kDirectT : 0;
    // + 0 turns the -0 of a negative input with |a'| < 1 into +0
    const double x = trunc(ldexp(a, s - tt)) + 0.0;
    in.x[q] = nz ? x : 0.0;
    in.t[q] = tt;
    huge |= tt > 0;
  }

  const int64_t slice_stride = lines_pad * kp;
  uint8_t *base = slices + kblocked(r, h0 + b * kRE, lines_pad);
  if (__any(huge))
    residue_moduli<true>(in, tab, N, nsq, nka, base, slice_stride);
  else
    residue_moduli<false>(in, tab, N, nsq, nka, base, slice_stride);
}

template <bool GROUPED, int SIDE>
__global__ __launch_bounds__(256) void k_residues(Problem P1, Group G) {
  __shared__ double tile[kQL * kRowLd];
  int64_t local;
  const Problem &P = *locate<GROUPED>(P1, G, blockIdx.x, local);
  const Operand &op = SIDE == 0 ? P.A : P.B;
  const int64_t base = SIDE == 0 ? 0 : P.w.lineB;
  const Dims d = family_dims(SIDE == 0 ? kFamResA : kFamResB, P);
  const int64_t bx = local % d.x, by = local / d.x;
  residues_tile(op, P.g.kp, SIDE == 0 ? P.g.mp : P.g.np, bx * kQL, by * kQK, P.w.shift + base,
                tables_of<GROUPED>(P1, G), P.g.N, P.g.nsq, P.g.nka,
                SIDE == 0 ? P.w.Asl : P.w.Bsl, tile);
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
  const int64_t blocks = grouped ? G->total : family_blocks(fam, *P);
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
    case kFamNormA: OZ2_Q2(k_bound_norm, 0) break;
    case kFamNormB: OZ2_Q2(k_bound_norm, 1) break;
    case kFamResA: OZ2_Q2(k_residues, 0) break;
    case kFamResB: OZ2_Q2(k_residues, 1) break;
    default: return hipErrorInvalidValue;
  }
#undef OZ2_Q
#undef OZ2_Q2
  return hipGetLastError();
}

}  // namespace oz2
