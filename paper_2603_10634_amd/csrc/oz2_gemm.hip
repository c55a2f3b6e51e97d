// FP8 E4M3 products on gfx950 MFMA (v_mfma_f32_32x32x64_f8f6f4), FP32
// accumulation.
//
//  * bound product: Cbar' = Abar Bbar (Section III-E); only the row and column
//    maxima of the FP32 result leave the kernel.
//  * residue products: per modulus the three digit products of Sections III-B
//    and III-C.  Digits are integers of magnitude <= 16, so over a chunk of
//    k <= 2^15 every partial sum is an integer of magnitude <= 2^24 and the
//    FP32 accumulation is exact (eq. error-free-FP8-matmult); the epilogue
//    combines the products and reduces them modulo p into int16 planes.
//  * INT8 arm (Section II): one product of the INT8 residues per modulus on
//    v_mfma_i32_32x32x32_i8, INT32 accumulation, the same wide loop.
//
// Layout: operand slices are k-blocked (see kblocked): one 64-k stage of a
// tile of 256 consecutive lines is 16 KB of contiguous memory.  The
// MFMA "A" operand is fed from B's slices (rows j) and the "B" operand from
// A's slices (rows i), so the accumulator holds D[j][i] = (A'B')_ij and each
// lane owns consecutive i of C's column-major planes.
//
// Workgroup: tile 256 (j) x 256 (i), 8 waves (the residue products; two per
// SIMD, each wave a 128 x 64 block as 4 x 2 MFMA tiles of 32 x 32) or 4 (the
// bound product; 128 x 128 each).  K advances 64 per stage through an LDS
// ring of S stages filled by direct global-to-LDS loads
// (global_load_lds_dwordx4) issued S - 1 stages ahead, so HBM/L2 latency
// hides behind S - 1 stages of MFMAs; no VGPRs stage the operands.  LDS rows
// are 64 B with the four 16 B chunks of row r XOR-swizzled by (r >> 2) & 3,
// which keeps the fragment reads (ds_read_b128) free of bank conflicts: gfx950
// serves a ds_read_b128 in passes of lanes 8p..8p+7 with 32+8p..32+8p+7, four
// cycles per instruction when each pass touches 16 different 16-byte bank
// groups (measured; the swizzle ((r >> 1) ^ (r >> 3)) & 3 took eight).
#include <string.h>

#include "oz2_internal.h"

namespace oz2 {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int TJ = 256;                  // tile rows (j, from B's slices)
constexpr int BK = 64;                   // k per stage (one MFMA step)
constexpr int ROWB = 64;                 // LDS bytes per tile row
constexpr int BSZ = TJ * ROWB;           // bytes of one B-side slice tile

__device__ __forceinline__ int swz(int r) { return (r >> 2) & 3; }

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8], vmcnt[5:4] at [15:14])
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14));
}
__device__ __forceinline__ void wait_lgkm0() {
  __builtin_amdgcn_s_waitcnt(0xF | (0x7 << 4) | (0x0 << 8) | (0x3 << 14));
}


__device__ __forceinline__ v16f mfma_f8(v8i a, v8i b, v16f c) {
  // cbsz = blgp = 0 selects E4M3 for both operands; zero scale operands give
  // the unscaled instruction
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// One 32 x 32 x 64 step of the single-product loop: an FP8 MFMA into FP32
// accumulators, or two INT8 MFMAs (32 k each) into INT32 accumulators.  The
// INT8 pair takes the low 16 bytes of every lane's 32-byte fragment first and
// the high 16 bytes second; both operands are split alike, so every byte of A
// still meets the byte of B with the same k and the sum covers all 64 k.
__device__ __forceinline__ v16f mma(v8i a, v8i b, v16f c) { return mfma_f8(a, b, c); }
__device__ __forceinline__ v16i mma(v8i a, v8i b, v16i c) {
  const v4i alo = __builtin_shufflevector(a, a, 0, 1, 2, 3);
  const v4i ahi = __builtin_shufflevector(a, a, 4, 5, 6, 7);
  const v4i blo = __builtin_shufflevector(b, b, 0, 1, 2, 3);
  const v4i bhi = __builtin_shufflevector(b, b, 4, 5, 6, 7);
  c = __builtin_amdgcn_mfma_i32_32x32x32_i8(alo, blo, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(ahi, bhi, c, 0, 0, 0);
}

// Operand fragment of a 32-row sub-tile: lane l holds row (l % 32) and the 32
// k bytes of logical chunks 2 (l / 32) and 2 (l / 32) + 1.  Both MFMA operands
// are read with the same k assignment, so the dot products pair matching k.
// row0 is always a multiple of 32, so the swizzle of row row0 + (l % 32) is
// that of l % 32: the per-lane byte offsets do not depend on row0, and every
// read is one per-lane address plus a constant (the ds_read immediate).
__device__ __forceinline__ v8i lds_frag(const uint8_t *tile, int row0, int tid) {
  const int lane = tid & 63;
  const int x = lane & 31, g = lane >> 5;
  const int f = swz(x);
  const uint8_t *row = tile + (row0 + x) * ROWB;
  const v4i lo = *(const v4i *)(row + 16 * ((2 * g) ^ f));
  const v4i hi = *(const v4i *)(row + 16 * ((2 * g + 1) ^ f));
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Values read from a problem descriptor or the tables through a generic
// pointer are wave-uniform but may sit in vector registers (a flat load could
// address per-lane private memory, so the compiler treats its result as
// divergent); the load issue below needs them in scalar registers.
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T *uni(T *p) {
  return (T *)(uintptr_t)uni((int64_t)(uintptr_t)p);
}

// One direct-to-LDS load: each lane fetches 16 B at `base` + `voff`; the
// wave's 64 chunks land contiguously at LDS byte address `lds_off` (held in
// M0).  It is issued from inline asm so that the compiler's wait-count
// analysis does not see an LDS write in flight (which would turn every
// LDS-read wait in the K-loop into a full drain); the K-loop waits for these
// loads itself with explicit vmcnt counts.  The compiler's hazard checks do
// not look inside inline asm, so the asm carries its own wait states: a VMEM
// instruction reading an SGPR that a VALU instruction wrote (for instance a
// v_readfirstlane the compiler places to move `base` into scalar registers,
// or an SGPR reload from a VGPR lane) needs 5, and the write of M0 before an
// LDS-DMA load needs 1.
__device__ __forceinline__ void dma16(const uint8_t *base, uint32_t voff, uint32_t lds_off) {
  asm volatile("s_nop 4\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(base),
               "{m0}"(lds_off)
               : "memory");
}

__device__ __forceinline__ uint32_t lds_offset(const uint8_t *p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const uint8_t *)p;
}

// Per-lane source offsets of the direct-to-LDS loads of a wave: ob[u] for
// its u-th 1 KB load (16 tile rows) on either side.  In the k-blocked layout
// the 16 rows of one load are 1 KB of contiguous memory; sB / sA are the
// bytes of one 64-k block of all lines of a side.
struct DmaOffsets {
  uint32_t ob[4];
  uint32_t lds_wave;  // 1024 * wave: this wave's first 1 KB in each tile
  int64_t sB, sA;
};

// s_waitcnt vmcnt(a L) for a run-time a in [0, A] (larger a: A L)
template <int L, int A>
__device__ __forceinline__ void wait_stages(int a) {
  if constexpr (A > 0) {
    if (a >= A) {
      wait_vm<A * L>();
      return;
    }
    wait_stages<L, A - 1>(a);
  } else {
    wait_vm<0>();
  }
}

// Values the epilogue needs are loaded with scalar loads, which complete out
// of order with LDS reads on the shared LGKM counter: while one is pending,
// every LDS wait in the K-loop degrades to a full drain.  Consuming them in an
// empty asm before the loop makes them resident first.
__device__ __forceinline__ void resident(int a, int b, int c, int d) {
  asm volatile("" ::"s"(a), "s"(b), "s"(c), "s"(d));
}
__device__ __forceinline__ void resident_ptr(const void *a, const void *b) {
  asm volatile("" ::"s"(a), "s"(b));
}

// Symmetric remainder of |v| < 2^31 modulo p, in [-floor(p/2), ceil(p/2) - 1].
// The float quotient estimate is within 1 of the rounded quotient.
__device__ __forceinline__ int smod_i32(int v, int p, float inv_p) {
  const int lo = -(p >> 1), hi = p - 1 - (p >> 1);
  const int q = (int)rintf((float)v * inv_p);
  int r = v - q * p;
  // branch-free corrections (sign masks rather than compare masks, which the
  // scheduler would otherwise keep live in scalar register pairs)
  r -= p & ((hi - r) >> 31);
  r += p & ((r - lo) >> 31);
  return r;
}

// ---------------------------------------------------------------------------
// Wide single-product tiles: 256 (j) x 256 (i) per workgroup, one product
// per pass into one accumulator per wave.  The residue products run 8 waves
// (two per SIMD, so one wave's MFMAs cover the other's barrier and LDS
// waits), each a 128 x 64 block as 4 x 2 MFMA tiles (128 AGPRs); the bound
// product runs 4 waves of 128 x 128 (256 AGPRs).  Per 64-k stage the
// workgroup moves 32 KB into LDS and reads at most 1.5 KB of fragments per
// MFMA, below the LDS rate.
// ---------------------------------------------------------------------------
constexpr int TIW = 256;                 // wide tile: i extent
constexpr int ASZW = TIW * ROWB;         // bytes of one A-side tile
constexpr int STAGEW = BSZ + ASZW;       // 32 KB per stage
constexpr int SW = 4;                    // ring slots
constexpr int LDS_RING = SW * STAGEW;    // 128 KB
static_assert(TIW == kGemmTIW && TJ == kGemmTJ && BK == kGemmBK, "tile shape");
// A wide workgroup has NW = 4 waves (one per SIMD, each 128 x 128) or 8 (two
// per SIMD, each 128 x 64, half the accumulator registers); per wave TB(NW)
// i blocks of 32 rows and LP(NW) 1 KB loads per side and stage.
constexpr int NW_RES = 8;                // the residue products
constexpr int NW_BOUND = 4;              // the bound product
template <int NW> constexpr int TB() { return 16 / NW; }
template <int NW> constexpr int LP() { return 16 / NW; }

// Lane offsets of the wide loads: wave w loads rows 16 (w + NWW u) .. + 15 of
// each side for u < LPW (both sides have 256 rows).
template <int NW>
__device__ __forceinline__ DmaOffsets dma_offsets_w(int64_t rowsB, int64_t rowsA, int tid) {
  constexpr int LPW = LP<NW>(), NWW = NW;
  DmaOffsets d;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rsub = lane >> 2, pc = lane & 3;
#pragma unroll
  for (int u = 0; u < LPW; ++u) {
    const int r = 16 * (wave + NWW * u) + rsub;
    d.ob[u] = (uint32_t)(r * 64) + 16u * (uint32_t)(pc ^ swz(r));
  }
  d.lds_wave = 1024u * (uint32_t)wave;
  d.sB = rowsB * 64;
  d.sA = rowsA * 64;
  return d;
}

// Load number idx (0 .. 2 LPW - 1) of a wide stage: the first LPW on the B
// side, the rest on the A side, each 1 KB = 16 rows.
template <int NW>
__device__ __forceinline__ void dma_one_w(int idx, const uint8_t *gB, const uint8_t *gA,
                                          const DmaOffsets &d, int64_t kofs, uint32_t slot) {
  constexpr int LPW = LP<NW>(), NWW = NW;
  const uint32_t w = slot + d.lds_wave;
  if (idx < LPW)
    dma16(gB + (kofs >> 6) * d.sB, d.ob[idx], w + idx * (NWW * 1024));
  else
    dma16(gA + (kofs >> 6) * d.sA, d.ob[idx - LPW], w + BSZ + (idx - LPW) * (NWW * 1024));
}

// The 2 LPW loads of a stage in four parts.
template <int NW, int Q>
__device__ __forceinline__ void dma_part_w(const uint8_t *gB, const uint8_t *gA,
                                           const DmaOffsets &d, int64_t kofs, uint32_t slot) {
  constexpr int PL = 2 * LP<NW>() / 4;
#pragma unroll
  for (int idx = PL * Q; idx < PL * Q + PL; ++idx) {
    dma_one_w<NW>(idx, gB, gA, d, kofs, slot);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One stage j of the wide loop (stage j sits in ring slot j % SW).  Wave w
// owns j rows 128 (w / (NWW / 2)) .. + 127 and i rows 32 TBW (w % (NWW / 2))
// .. + 32 TBW - 1; ACC is v16f (FP8 products) or v16i (INT8 products).
// Schedule, over the four block rows tj of TBW MFMAs each:
//   tj = 0..2: the B-side fragment of block row tj + 1 is read, then the
//     MFMAs of block row tj issue with part tj + 1 of the loads of stage
//     j + SW - 1 after the first of them;
//   barrier B_j: before it each wave waits until its own loads of stage j + 1
//     have landed and its LDS reads of stage j are complete, so after it
//     stage j + 1 is readable by all and slot j % SW is free;
//   tj = 3: its MFMAs issue with part 0 of the loads of stage j + SW (into
//     slot j % SW) and the reads of stage j + 1's A-side fragments and first
//     B-side block row between them, so that LDS latency and the barrier hide
//     behind MFMAs already in registers.
template <int NW, bool STEADY, bool CHAIN, class ACC>
__device__ __forceinline__ void stage_iter_w(int j, int nk, const uint8_t *gB, const uint8_t *gA,
                                             const uint8_t *gBn, const uint8_t *gAn,
                                             const DmaOffsets &d, int64_t kbeg,
                                             const uint8_t *lds, uint32_t ring,
                                             const v8i (&fa)[TB<NW>()], v8i (&fan)[TB<NW>()],
                                             v8i (&fb)[4], ACC (&acc)[4][TB<NW>()], int tid) {
  constexpr int TBW = TB<NW>(), NWW = NW;
  constexpr int L = 2 * LP<NW>();
  const int wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  const uint8_t *cur = lds + (j % SW) * STAGEW;
  // STEADY: j + SW < nk, so every load and read below exists.  CHAIN: the
  // loads of stages past nk - 1 fetch the next pass's first stages (from gBn,
  // gAn; nk is a multiple of SW, so into the slots its own prologue would
  // use), exactly as a steady stage would, so the waits are the steady ones
  const bool ld_prev = STEADY || CHAIN || j + SW - 1 < nk;
  const bool ld_next = STEADY || CHAIN || j + SW < nk;
  const bool rd_next = STEADY || j + 1 < nk;
  const bool prev_here = STEADY || j + SW - 1 < nk;
  const bool next_here = STEADY || j + SW < nk;
  const uint8_t *gBp = prev_here ? gB : gBn, *gAp = prev_here ? gA : gAn;
  const uint8_t *gBx = next_here ? gB : gBn, *gAx = next_here ? gA : gAn;
  const int64_t kofs_prev = kbeg + (int64_t)(j + SW - 1 - (prev_here ? 0 : nk)) * BK;
  const int64_t kofs_next = kbeg + (int64_t)(j + SW - (next_here ? 0 : nk)) * BK;
  const uint32_t slot_prev = ring + ((j + SW - 1) % SW) * STAGEW;
#pragma unroll
  for (int tj = 0; tj < 3; ++tj) {
    fb[tj + 1] = lds_frag(cur, wj * 128 + (tj + 1) * 32, tid);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
      acc[tj][ti] = mma(fb[tj], fa[ti], acc[tj][ti]);
      __builtin_amdgcn_sched_barrier(0);
      if (ti == 0 && ld_prev) {
        if (tj == 0) dma_part_w<NW, 1>(gBp, gAp, d, kofs_prev, slot_prev);
        if (tj == 1) dma_part_w<NW, 2>(gBp, gAp, d, kofs_prev, slot_prev);
        if (tj == 2) dma_part_w<NW, 3>(gBp, gAp, d, kofs_prev, slot_prev);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  wait_lgkm0();
  if (STEADY || (CHAIN && rd_next))
    wait_vm<(SW - 2) * L>();
  else if (rd_next)
    wait_stages<L, SW - 2>(nk - 2 - j);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  const uint8_t *nxt = lds + ((j + 1) % SW) * STAGEW;
#pragma unroll
  for (int ti = 0; ti < TBW; ++ti) {
    acc[3][ti] = mma(fb[3], fa[ti], acc[3][ti]);
    __builtin_amdgcn_sched_barrier(0);
    if (ti == 0 && ld_next)
      dma_part_w<NW, 0>(gBx, gAx, d, kofs_next, ring + (j % SW) * STAGEW);
    if (rd_next) {
      // the next stage's fragments: the A side after MFMA 0, then B block 0
      if (ti == 0) {
#pragma unroll
        for (int t = 0; t < TBW; ++t) fan[t] = lds_frag(nxt + BSZ, wi * 32 * TBW + t * 32, tid);
      }
      if (ti == TBW - 1) fb[0] = lds_frag(nxt, wj * 128, tid);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// acc += A B over nk stages of 64 k for one wide tile; gB / gA point at row
// j0 / i0 of one B-side / A-side slice.  Passes of one tile over the same k
// range can be chained: with CHAIN_OUT the last stages also load the first
// stages of the next pass (gBn, gAn), which the next pass's loop, with
// CHAIN_IN, then finds in flight instead of issuing them itself; the fold
// between the passes runs while they land.
template <int NW, bool CHAIN_IN = false, bool CHAIN_OUT = false, class ACC>
__device__ __forceinline__ void kloop_w(const uint8_t *gB, const uint8_t *gA, int64_t rowsB,
                                        int64_t rowsA, int64_t kbeg, int nk, uint8_t *lds,
                                        ACC (&acc)[4][TB<NW>()], int tid,
                                        const uint8_t *gBn = nullptr,
                                        const uint8_t *gAn = nullptr) {
  constexpr int TBW = TB<NW>(), NWW = NW;
  constexpr int L = 2 * LP<NW>();
  const int wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  const DmaOffsets d = dma_offsets_w<NW>(rowsB, rowsA, tid);
  const uint32_t ring = lds_offset(lds);
  if (!CHAIN_IN) {
#pragma unroll
    for (int t = 0; t < SW - 1; ++t)
      if (t < nk) {
#pragma unroll
        for (int idx = 0; idx < L; ++idx)
          dma_one_w<NW>(idx, gB, gA, d, kbeg + (int64_t)t * BK, ring + t * STAGEW);
      }
    if (SW - 1 < nk)
      dma_part_w<NW, 0>(gB, gA, d, kbeg + (int64_t)(SW - 1) * BK, ring + (SW - 1) * STAGEW);
  }
  if (SW - 1 < nk)
    wait_vm<(SW - 2) * L + L / 4>();
  else
    wait_stages<L, SW - 2>(nk - 1);
  __builtin_amdgcn_s_barrier();
  v8i fa0[TBW], fa1[TBW], fb[4];
#pragma unroll
  for (int ti = 0; ti < TBW; ++ti) fa0[ti] = lds_frag(lds + BSZ, wi * 32 * TBW + ti * 32, tid);
  fb[0] = lds_frag(lds, wj * 128, tid);
  // nk is a multiple of 4 (k is padded to 256): two stages per trip, no tail;
  // the trips whose stages all load a later stage run without the checks
  int j = 0;
  for (; j + 1 + SW < nk; j += 2) {
    stage_iter_w<NW, true, false>(j, nk, gB, gA, gB, gA, d, kbeg, lds, ring, fa0, fa1, fb, acc,
                                  tid);
    stage_iter_w<NW, true, false>(j + 1, nk, gB, gA, gB, gA, d, kbeg, lds, ring, fa1, fa0, fb,
                                  acc, tid);
  }
  for (; j < nk; j += 2) {
    stage_iter_w<NW, false, CHAIN_OUT>(j, nk, gB, gA, gBn, gAn, d, kbeg, lds, ring, fa0, fa1, fb,
                                       acc, tid);
    stage_iter_w<NW, false, CHAIN_OUT>(j + 1, nk, gB, gA, gBn, gAn, d, kbeg, lds, ring, fa1, fa0,
                                       fb, acc, tid);
  }
  __builtin_amdgcn_s_barrier();
}

// Keeps the accumulator tiles in AGPRs at this point (an empty asm with
// AGPR in/out operands), so the register allocator does not move the whole
// accumulator to VGPRs around the folds between passes.
template <class ACC, int T>
__device__ __forceinline__ void pin_agpr(ACC (&acc)[4][T]) {
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < T; ++ti) asm volatile("" : "+a"(acc[tj][ti]));
}

// acc = mul acc (mod p), reduced to |acc| <= p/2 + 2, one 16-value MFMA tile
// at a time, in FP32: for an exact integer |x| < 2^24 the quotient estimate
// rint(x p^-1) misses x / p by less than 2 / p + 1/2, so x - q p (one exact
// fused multiply-add) has |x - q p| <= p/2 + 2; times |mul| <= 256 it stays
// below 2^17 and is reduced the same way.  Any representative that small
// keeps the next pass's FP32 accumulation exact (below 2^24); the epilogue
// takes the symmetric remainder.
template <int TBW>
__device__ __forceinline__ void fold_w(v16f (&acc)[4][TBW], int mul, int p, float inv) {
  const float pf = (float)p, mf = (float)mul;
  pin_agpr(acc);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
      v16f t16;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float x = acc[tj][ti][v];
        const float y = fmaf(-rintf(x * inv), pf, x) * mf;
        t16[v] = fmaf(-rintf(y * inv), pf, y);
      }
      acc[tj][ti] = t16;
      asm volatile("" : "+a"(acc[tj][ti]));
      __builtin_amdgcn_sched_barrier(0);
    }
}

// One 256 x 256 tile (j0.., i0..) of Karatsuba modulus l (s = 16) over k in
// [kbeg, kbeg + 64 nk), three single-product passes in one accumulator.
// The digit products C1 = A1 B1, C2 = A2 B2, C3 = A3 B3 combine to
// 240 C1 - 15 C2 + 16 C3 (eq. C'-Karatsuba) = c (b (a X + Y) + Z) (mod p),
// with the passes (X, Y, Z) and multipliers from the tables:
//   (C1, C3, C2), a = 15, b = -16/15, c = -15  (p coprime to 15), or
//   (C1, C2, C3), a = -16, b = -15/16, c = 16  (other odd p):
//   pass 1: acc = X;         fold: acc = smod(a smod(acc))
//   pass 2: acc += Y;        fold: acc = smod(b smod(acc))
//   pass 3: acc += Z;        result smod(c acc)
// Every fold leaves |acc| <= p/2 <= 256, so the FP32 accumulation of each
// pass stays an exact integer below 2^24.
template <int NW>
__device__ __forceinline__ void karatsuba_tile_w(const uint8_t *Asl, const uint8_t *Bsl,
                                                 int16_t *__restrict__ planes,
                                                 const Tables *__restrict__ tab, int64_t mp,
                                                 int64_t np, int64_t kp, int64_t kbeg, int nk,
                                                 int accumulate, int l, int64_t i0, int64_t j0,
                                                 uint8_t *lds, int tid) {
  const int sl0 = (int)uni(tab->slice0[l]);
  const int p = (int)uni(tab->p[l]);
  const float inv = __int_as_float((int)uni(__float_as_int(tab->inv_p[l])));
  const int mul_a = (int)uni(tab->kfold[l][0]);
  const int mul_b = (int)uni(tab->kfold[l][1]);
  const int mul_c = (int)uni(tab->kfold[l][2]);
  const int second = (int)uni(tab->kfold[l][3]);  // slice of pass 2 (pass 3: 3 - second)
  resident(sl0, p, __float_as_int(inv), mul_a);
  resident(mul_b, mul_c, second, second);
  resident_ptr(planes, planes);
  resident(accumulate, accumulate, accumulate, accumulate);
  const int64_t sA = mp * kp, sB = np * kp;
  const uint8_t *A0 = Asl + (int64_t)sl0 * sA + i0 * 64;
  const uint8_t *B0 = Bsl + (int64_t)sl0 * sB + j0 * 64;

  constexpr int NWW = NW, TBW = TB<NW>();
  v16f acc[4][TBW];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tj][ti][v] = 0.0f;

  pin_agpr(acc);
  const int third = 3 - second;
  kloop_w<NWW, false, true>(B0, A0, np, mp, kbeg, nk, lds, acc, tid, B0 + second * sB,
                            A0 + second * sA);                                      // X = C1
  fold_w(acc, mul_a, p, inv);
  kloop_w<NWW, true, true>(B0 + second * sB, A0 + second * sA, np, mp, kbeg, nk, lds, acc, tid,
                           B0 + third * sB, A0 + third * sA);                       // + Y
  fold_w(acc, mul_b, p, inv);
  kloop_w<NWW, true, false>(B0 + third * sB, A0 + third * sA, np, mp, kbeg, nk, lds, acc,
                            tid);                                                   // + Z

  const int lane = tid & 63, wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  int16_t *out = planes + (int64_t)l * np * mp;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int r = smod_i32(mul_c * (int)acc[tj][ti][v], p, inv);
        const int64_t i = i0 + wi * 32 * TBW + ti * 32 + (lane & 31);
        const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        int16_t *dst = out + j * mp + i;
        if (accumulate) r = smod_i32(r + (int)*dst, p, inv);
        *dst = (int16_t)r;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
}

// acc = m (acc mods q) mods r, one 16-value MFMA tile at a time, in FP32,
// with the reductions of fold_w (x - rint(x q^-1) q, exact); 1/r = 0 skips
// the second reduction.
template <int TBW>
__device__ __forceinline__ void fold_g(v16f (&acc)[4][TBW], float q, float inv_q, float m,
                                       float r, float inv_r) {
  pin_agpr(acc);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
      v16f t16;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float x = acc[tj][ti][v];
        const float y = fmaf(-rintf(x * inv_q), q, x) * m;
        t16[v] = fmaf(-rintf(y * inv_r), r, y);
      }
      acc[tj][ti] = t16;
      asm volatile("" : "+a"(acc[tj][ti]));
      __builtin_amdgcn_sched_barrier(0);
    }
}

// acc = s (acc mod s) for a square modulus p = s^2, one 16-value MFMA tile at
// a time, in FP32: the first pass sums X = A1 B2 + A2 B1, of which only
// s X mod s^2 = s (X mod s) matters.  As in fold_w, x - rint(x s^-1) s is an
// exact representative with |.| <= s/2 + 2, so |acc| <= s (s/2 + 2) < 2^10.
template <int TBW>
__device__ __forceinline__ void fold_s(v16f (&acc)[4][TBW], int s, float inv_s) {
  const float sf = (float)s;
  pin_agpr(acc);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
      v16f t16;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float x = acc[tj][ti][v];
        t16[v] = fmaf(-rintf(x * inv_s), sf, x) * sf;
      }
      acc[tj][ti] = t16;
      asm volatile("" : "+a"(acc[tj][ti]));
      __builtin_amdgcn_sched_barrier(0);
    }
}

// One 256 x 256 tile (j0.., i0..) of square modulus l (p = s^2, Section
// III-C) over k in [kbeg, kbeg + 64 nk), three single-product passes in one
// accumulator.  With A = A1 s + A2 and B = B1 s + B2, A B = s^2 A1 B1 +
// s (A1 B2 + A2 B1) + A2 B2 (eq. 3matmult-notKaratsuba), and the first term
// vanishes modulo s^2:
//   passes 1, 2: acc = A1 B2 + A2 B1;  fold: acc = s (acc mod s)
//   pass 3:      acc += A2 B2;         result smod(acc)
// The residue has |u| <= s^2 / 2 and s <= 33, so |A1| = |round(u / s)| <= 16
// and |A2| <= s / 2, i.e. <= 16: over a k chunk of at most 2^15 the first two
// passes sum to at most 2 (16^2) 2^15 = 2^24 in magnitude, the third adds at
// most 2^23 to |acc| < 2^10, and every partial sum is an exact FP32 integer.
template <int NW>
__device__ __forceinline__ void square_tile_w(const uint8_t *Asl, const uint8_t *Bsl,
                                              int16_t *__restrict__ planes,
                                              const Tables *__restrict__ tab, int64_t mp,
                                              int64_t np, int64_t kp, int64_t kbeg, int nk,
                                              int accumulate, int l, int64_t i0, int64_t j0,
                                              uint8_t *lds, int tid) {
  const int sl0 = (int)uni(tab->slice0[l]);
  const int p = (int)uni(tab->p[l]);
  const float inv = __int_as_float((int)uni(__float_as_int(tab->inv_p[l])));
  const int s = (int)uni(tab->s[l]);
  const float inv_s = __int_as_float((int)uni(__float_as_int(tab->inv_s[l])));
  resident(sl0, p, __float_as_int(inv), s);
  resident(__float_as_int(inv_s), s, s, s);
  resident_ptr(planes, planes);
  resident(accumulate, accumulate, accumulate, accumulate);
  const int64_t sA = mp * kp, sB = np * kp;
  const uint8_t *A0 = Asl + (int64_t)sl0 * sA + i0 * 64;
  const uint8_t *B0 = Bsl + (int64_t)sl0 * sB + j0 * 64;

  constexpr int NWW = NW, TBW = TB<NW>();
  v16f acc[4][TBW];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tj][ti][v] = 0.0f;

  pin_agpr(acc);
  kloop_w<NWW, false, true>(B0 + sB, A0, np, mp, kbeg, nk, lds, acc, tid, B0,
                            A0 + sA);                                               // A1 B2
  pin_agpr(acc);
  kloop_w<NWW, true, true>(B0, A0 + sA, np, mp, kbeg, nk, lds, acc, tid, B0 + sB,
                           A0 + sA);                                                // + A2 B1
  fold_s(acc, s, inv_s);
  kloop_w<NWW, true, false>(B0 + sB, A0 + sA, np, mp, kbeg, nk, lds, acc, tid);     // + A2 B2

  const int lane = tid & 63, wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  int16_t *out = planes + (int64_t)l * np * mp;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int r = smod_i32((int)acc[tj][ti][v], p, inv);
        const int64_t i = i0 + wi * 32 * TBW + ti * 32 + (lane & 31);
        const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        int16_t *dst = out + j * mp + i;
        if (accumulate) r = smod_i32(r + (int)*dst, p, inv);
        *dst = (int16_t)r;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
}

// One 256 x 256 tile (j0.., i0..) of INT8 modulus l (Section II) over k in
// [kbeg, kbeg + 64 nk): the one product of the INT8 residues, accumulated in
// INT32 (|u| <= 128, so a chunk of k <= 2^15 sums to at most 2^29), then
// reduced modulo p.
template <int NW>
__device__ __forceinline__ void int8_tile_w(const uint8_t *Asl, const uint8_t *Bsl,
                                            int16_t *__restrict__ planes,
                                            const Tables *__restrict__ tab, int64_t mp,
                                            int64_t np, int64_t kp, int64_t kbeg, int nk,
                                            int accumulate, int l, int64_t i0, int64_t j0,
                                            uint8_t *lds, int tid) {
  const int sl0 = (int)uni(tab->slice0[l]);
  const int p = (int)uni(tab->p[l]);
  const float inv = __int_as_float((int)uni(__float_as_int(tab->inv_p[l])));
  resident(sl0, p, __float_as_int(inv), p);
  resident_ptr(planes, planes);
  resident(accumulate, accumulate, accumulate, accumulate);
  const uint8_t *A0 = Asl + (int64_t)sl0 * mp * kp + i0 * 64;
  const uint8_t *B0 = Bsl + (int64_t)sl0 * np * kp + j0 * 64;

  constexpr int NWW = NW, TBW = TB<NW>();
  v16i acc[4][TBW];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tj][ti][v] = 0;
  pin_agpr(acc);
  kloop_w<NWW>(B0, A0, np, mp, kbeg, nk, lds, acc, tid);
  pin_agpr(acc);

  const int lane = tid & 63, wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  int16_t *out = planes + (int64_t)l * np * mp;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int r = smod_i32(acc[tj][ti][v], p, inv);
        const int64_t i = i0 + wi * 32 * TBW + ti * 32 + (lane & 31);
        const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        int16_t *dst = out + j * mp + i;
        if (accumulate) r = smod_i32(r + (int)*dst, p, inv);
        *dst = (int16_t)r;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
}

// Residue products of one problem, 256 x 256 tiles: KIND 0 over the square
// moduli (l = z mod nsq), 1 over the Karatsuba moduli (l = nsq + z mod nka),
// 2 over the INT8 moduli (l = nsq + nka + z mod n8).  The workgroup covers k
// part z / (moduli of the kind) of P.parts and writes that part's copy of the
// planes; the host makes every part at most kChunkK long.
template <int KIND>
__global__ __launch_bounds__(64 * NW_RES, 1) void k_residue_gemm(Problem P) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[LDS_RING];
  const Geometry &g = P.g;
  const Dims d = family_dims(KIND == 0 ? kFamGemmSq : (KIND == 1 ? kFamGemmKa : kFamGemmI8), P);
  const Dims c = decode_block(d, blockIdx.x);
  const int64_t mp = uni(g.mp), np = uni(g.np), kp = uni(g.kp);
  const int parts = (int)uni((int64_t)P.parts);
  const int64_t nz = d.z / parts;
  const int part = (int)uni(c.z / nz);
  const int l = (int)uni((KIND == 0 ? 0 : (KIND == 1 ? g.nsq : g.nsq + g.nka)) + c.z % nz);
  int64_t k0, k1;
  part_range(kp, parts, part, &k0, &k1);
  const int nk = (int)uni((k1 - k0) / BK);
  k0 = uni(k0);
  int16_t *planes = uni(P.w.planes) + uni((int64_t)part * g.N) * mp * np;
  const int tid = threadIdx.x;
  if (KIND == 0)
    square_tile_w<NW_RES>(uni(P.w.Asl), uni(P.w.Bsl), planes, uni(P.tab), mp, np, kp, k0, nk, 0,
                          l, uni(c.x * TIW), uni(c.y * TJ), lds, tid);
  else if (KIND == 1)
    karatsuba_tile_w<NW_RES>(uni(P.w.Asl), uni(P.w.Bsl), planes, uni(P.tab), mp, np, kp, k0, nk,
                             0, l, uni(c.x * TIW), uni(c.y * TJ), lds, tid);
  else
    int8_tile_w<NW_RES>(uni(P.w.Asl), uni(P.w.Bsl), planes, uni(P.tab), mp, np, kp, k0, nk, 0, l,
                        uni(c.x * TIW), uni(c.y * TJ), lds, tid);
}

// One 256 x 256 tile of any FP8 modulus (square or Karatsuba) as three
// single-product passes with two folds, every step from the tables:
//   pass 1: acc = D(a1, b1);   fold: acc = m1 (acc mods q1), then mods r1
//   pass 2: acc += D(a2, b2);  fold: acc = m2 (acc mods q2), then mods r2
//   pass 3: acc += D(a3, b3);  result smod(m3 acc, p)
// where D(a, b) is the product of A's digit slice a and B's slice b.
//   square p = s^2 (as square_tile_w): passes (1, 2), (2, 1), (2, 2); the
//     first fold reduces modulo p (X mod s is all that matters), the second
//     is s (acc mods s) with no further reduction; m3 = 1;
//   Karatsuba (as karatsuba_tile_w): passes X, Y, Z, folds a, b modulo p
//     (each followed by a reduction modulo p), m3 = c.
// A fold "then mods r" with no reduction uses 1/r = 0.  Every fold leaves
// |acc| <= 2^10, so each pass's FP32 accumulation stays exact.
template <int NW>
__device__ __forceinline__ void fp8_tile_w(const uint8_t *Asl, const uint8_t *Bsl,
                                           int16_t *__restrict__ planes,
                                           const Tables *__restrict__ tab, int64_t mp,
                                           int64_t np, int64_t kp, int64_t kbeg, int nk,
                                           int accumulate, int l, int64_t i0, int64_t j0,
                                           uint8_t *lds, int tid) {
  const int sl0 = (int)uni(tab->slice0[l]);
  const int p = (int)uni(tab->p[l]);
  const float inv = __int_as_float((int)uni(__float_as_int(tab->inv_p[l])));
  const bool square = uni(tab->kind[l]) == 0;
  const int s = (int)uni(tab->s[l]);
  const float inv_s = __int_as_float((int)uni(__float_as_int(tab->inv_s[l])));
  const int second = square ? 0 : (int)uni(tab->kfold[l][3]);
  // passes: (A slice, B slice)
  const int a1 = 0, b1 = square ? 1 : 0;
  const int a2 = square ? 1 : second, b2 = square ? 0 : second;
  const int a3 = square ? 1 : 3 - second, b3 = square ? 1 : 3 - second;
  // folds
  const float q2 = square ? (float)s : (float)p, iq2 = square ? inv_s : inv;
  const float m1 = square ? 1.0f : (float)uni(tab->kfold[l][0]);
  const float m2 = square ? (float)s : (float)uni(tab->kfold[l][1]);
  const float ir2 = square ? 0.0f : inv;
  const int m3 = square ? 1 : (int)uni(tab->kfold[l][2]);
  resident(sl0, p, __float_as_int(inv), s);
  resident(__float_as_int(inv_s), second, m3, m3);
  resident_ptr(planes, planes);
  resident(accumulate, accumulate, accumulate, accumulate);
  const int64_t sA = mp * kp, sB = np * kp;
  const uint8_t *A0 = Asl + (int64_t)sl0 * sA + i0 * 64;
  const uint8_t *B0 = Bsl + (int64_t)sl0 * sB + j0 * 64;

  constexpr int NWW = NW, TBW = TB<NW>();
  v16f acc[4][TBW];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tj][ti][v] = 0.0f;

  pin_agpr(acc);
  kloop_w<NWW, false, true>(B0 + b1 * sB, A0 + a1 * sA, np, mp, kbeg, nk, lds, acc, tid,
                            B0 + b2 * sB, A0 + a2 * sA);
  fold_g(acc, (float)p, inv, m1, (float)p, inv);
  kloop_w<NWW, true, true>(B0 + b2 * sB, A0 + a2 * sA, np, mp, kbeg, nk, lds, acc, tid,
                           B0 + b3 * sB, A0 + a3 * sA);
  fold_g(acc, q2, iq2, m2, (float)p, ir2);
  kloop_w<NWW, true, false>(B0 + b3 * sB, A0 + a3 * sA, np, mp, kbeg, nk, lds, acc, tid);

  const int lane = tid & 63, wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  int16_t *out = planes + (int64_t)l * np * mp;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int r = smod_i32(m3 * (int)acc[tj][ti][v], p, inv);
        const int64_t i = i0 + wi * 32 * TBW + ti * 32 + (lane & 31);
        const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        int16_t *dst = out + j * mp + i;
        if (accumulate) r = smod_i32(r + (int)*dst, p, inv);
        *dst = (int16_t)r;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
}

// The residue products of a whole batch in one launch: each workgroup takes
// the next item of the work list (tile x modulus x k part of one problem,
// longest first) until the list is exhausted; the k chunks of an item run in
// order inside the workgroup, accumulating into its plane copy.  INT8 = the
// INT8 arm's products, else the FP8 moduli of either kind.  The last
// workgroup to finish clears the counters for the next launch, so the launch
// needs no memset and replays from a graph.
template <int NW, bool INT8>
__global__ __launch_bounds__(64 * NW, 1) void k_residue_persistent(WorkList W) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[LDS_RING];
  __shared__ uint32_t item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(&W.counters[0], 1u);
    __syncthreads();
    const int64_t it = (int64_t)__builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();
    if (it >= W.count) break;
    const ProductItem *I = uni(W.items) + it;
    const Problem &P = uni(W.probs)[(int)uni((int64_t)I->prob)];
    const int64_t mp = uni(P.g.mp), np = uni(P.g.np), kp = uni(P.g.kp);
    const int l = (int)uni((int64_t)I->l);
    const int64_t k0 = uni((int64_t)I->k0), k1 = uni((int64_t)I->k1);
    const int64_t i0 = uni((int64_t)I->tx * TIW), j0 = uni((int64_t)I->ty * TJ);
    int16_t *planes = uni(P.w.planes) + uni((int64_t)I->part * P.g.N) * mp * np;
    for (int64_t kb = k0; kb < k1; kb += kChunkK) {
      const int64_t len = k1 - kb < kChunkK ? k1 - kb : kChunkK;
      // the thread index, opaque to the compiler once per chunk: the
      // epilogue's addresses derived from it are then formed after the
      // k-loop instead of being hoisted above it and kept live (spilled)
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      if (INT8)
        int8_tile_w<NW>(uni(P.w.Asl), uni(P.w.Bsl), planes, uni(P.tab), mp, np, kp, kb,
                        (int)(len / BK), kb > k0 ? 1 : 0, l, i0, j0, lds, tid);
      else
        fp8_tile_w<NW>(uni(P.w.Asl), uni(P.w.Bsl), planes, uni(P.tab), mp, np, kp, kb,
                       (int)(len / BK), kb > k0 ? 1 : 0, l, i0, j0, lds, tid);
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&W.counters[1], 1u) == gridDim.x - 1) {
      atomicExch(&W.counters[0], 0u);
      atomicExch(&W.counters[1], 0u);
    }
  }
}

// Line maxima of one 256 x 256 tile (j0.., i0..) of the bound product held in
// acc (the layout of the wide tile loop): row maxima into rmaxA, column maxima
// into rmaxB, by atomic maxima over the tiles.
__device__ __forceinline__ void bound_maxima(const v16f (&acc)[4][TB<NW_BOUND>()],
                                             uint32_t *__restrict__ rmaxA,
                                             uint32_t *__restrict__ rmaxB, int64_t i0,
                                             int64_t j0, int tid) {
  constexpr int NWW = NW_BOUND, TBW = TB<NW_BOUND>();
  const int lane = tid & 63, wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  // maxima over j of each column i (row maxima of Abar Bbar, for mu)
#pragma unroll
  for (int ti = 0; ti < TBW; ++ti) {
    float m = 0.0f;
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int v = 0; v < 16; ++v) m = fmaxf(m, acc[tj][ti][v]);
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    if (lane < 32)
      atomicMax(&rmaxA[i0 + wi * 32 * TBW + ti * 32 + lane], __float_as_uint(m));
  }
  // maxima over i of each row j (column maxima of Abar Bbar, for nu)
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float m = acc[tj][0][v];
#pragma unroll
      for (int ti = 1; ti < TBW; ++ti) m = fmaxf(m, acc[tj][ti][v]);
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
      if ((lane & 31) == 0) {
        const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        atomicMax(&rmaxB[j], __float_as_uint(m));
      }
    }
}

// Part sums of the split bound product: value q of thread t of tile `tile`
// of part `part` at ((part * tiles + tile) * kBoundVals + q) * threads + t,
// so that each access of a wave covers 256 consecutive bytes.
constexpr int kBoundThreads = 64 * NW_BOUND;
constexpr int kBoundVals = 4 * TB<NW_BOUND>() * 16;
static_assert(4 * TB<NW_BOUND>() == 16, "k_bound_reduce's grid assumes 16 MFMA blocks per wave");

__device__ __forceinline__ int64_t bound_part_at(int64_t part, int64_t tiles, int64_t tile,
                                                 int q, int tid) {
  return ((part * tiles + tile) * kBoundVals + q) * kBoundThreads + tid;
}

// One 256 x 256 tile of the bound product Abar Bbar over k in [kbeg, kbeg +
// 64 nk) (wide single-product loop; FP32 accumulation in one fixed k order,
// so the result does not depend on the tiling): its line maxima, or with
// part_out its FP32 sums stored for k_bound_reduce.
__device__ __forceinline__ void bound_tile(const uint8_t *Abar, const uint8_t *Bbar, int64_t mp,
                                           int64_t np, int64_t kbeg, int nk,
                                           uint32_t *__restrict__ rmaxA,
                                           uint32_t *__restrict__ rmaxB,
                                           float *__restrict__ part_out, int64_t i0, int64_t j0,
                                           uint8_t *lds, int tid) {
  constexpr int NWW = NW_BOUND, TBW = TB<NW_BOUND>();
  v16f acc[4][TBW];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < TBW; ++ti)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tj][ti][v] = 0.0f;
  resident_ptr(rmaxA, rmaxB);
  pin_agpr(acc);
  kloop_w<NWW>(Bbar + j0 * 64, Abar + i0 * 64, np, mp, kbeg, nk, lds, acc, tid);
  pin_agpr(acc);
  if (part_out) {
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int ti = 0; ti < TBW; ++ti)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          part_out[(int64_t)((tj * TBW + ti) * 16 + v) * kBoundThreads + tid] = acc[tj][ti][v];
    return;
  }
  bound_maxima(acc, rmaxA, rmaxB, i0, j0, tid);
}

template <bool GROUPED>
__global__ __launch_bounds__(64 * NW_BOUND, 1) void k_bound_gemm(Problem P1, Group G) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[LDS_RING];
  const int64_t total = GROUPED ? G.total : (int64_t)gridDim.x;
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    int64_t local;
    const Problem &P = *locate<GROUPED>(P1, G, b, local);
    const Geometry &g = P.g;
    const Dims d = family_dims(kFamBgemm, P);
    const Dims c = decode_block(d, local);
    const int64_t mp = uni(g.mp), np = uni(g.np), kp = uni(g.kp);
    uint32_t *rmax = uni(P.w.rmax);
    // a split product (single problems only): part c.z of P.bparts
    const int parts = GROUPED ? 1 : (int)uni((int64_t)P.bparts);
    int64_t k0 = 0, k1 = kp;
    float *part_out = nullptr;
    if (!GROUPED && parts > 1) {
      part_range(kp, parts, (int)c.z, &k0, &k1);
      const int64_t tiles = d.x * d.y;
      part_out = uni(P.w.bpart) + bound_part_at(c.z, tiles, c.y * d.x + c.x, 0, 0);
    }
    bound_tile(uni(P.w.Abar), uni(P.w.Bbar), mp, np, uni(k0), (int)uni((k1 - k0) / BK), rmax,
               rmax + mp, part_out, uni(c.x * TIW), uni(c.y * TJ), lds, threadIdx.x);
  }
}

// Split bound product: per tile and MFMA block (tj, ti) of every wave, the
// FP32 sum of its parts in part order, then that block's line maxima.  Block
// z of the launch takes tile z / (4 TBW) and (tj, ti) from z mod (4 TBW), so
// that the launch has 4 TBW workgroups per tile.
__global__ __launch_bounds__(64 * NW_BOUND) void k_bound_reduce(Problem P) {
  constexpr int TBW = TB<NW_BOUND>(), NWW = NW_BOUND;
  const Dims d = family_dims(kFamBgemm, P);
  const int64_t tiles = d.x * d.y;
  const int64_t tile = blockIdx.x / (4 * TBW);
  const int sub = (int)(blockIdx.x % (4 * TBW));
  const int tj = sub / TBW, ti = sub % TBW;
  const int parts = P.bparts;
  const int tid = threadIdx.x;
  const float *src = P.w.bpart + bound_part_at(0, tiles, tile, sub * 16, tid);
  const int64_t part_stride = tiles * kBoundVals * kBoundThreads;
  float acc[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = src[v * kBoundThreads];
#pragma unroll 4
  for (int q = 1; q < parts; ++q) {
    const float *s = src + q * part_stride;
    float x[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) x[v] = s[v * kBoundThreads];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] += x[v];
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int wj = wave / (NWW / 2), wi = wave % (NWW / 2);
  const int64_t i0 = (tile % d.x) * TIW, j0 = (tile / d.x) * TJ;
  uint32_t *rmaxA = P.w.rmax, *rmaxB = P.w.rmax + P.g.mp;
  // row maxima (rows i of this block: one per lane % 32)
  float m = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) m = fmaxf(m, acc[v]);
  m = fmaxf(m, __shfl_xor(m, 32, 64));
  if (lane < 32) atomicMax(&rmaxA[i0 + wi * 32 * TBW + ti * 32 + lane], __float_as_uint(m));
  // column maxima (columns j: one per value v and lane / 32)
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    float c = acc[v];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) c = fmaxf(c, __shfl_xor(c, off, 64));
    if ((lane & 31) == 0) {
      const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      atomicMax(&rmaxB[j], __float_as_uint(c));
    }
  }
}

}  // namespace

hipError_t launch_gemm_persistent(int nw, bool int8, const WorkList &W, int64_t grid,
                                  hipStream_t st) {
  if (W.count <= 0) return hipSuccess;
  if (grid > W.count) grid = W.count;
  if (grid <= 0 || grid > 0x7FFFFFFFll || W.count > 0xFFFFFFFFll) return hipErrorInvalidValue;
  const dim3 gr((unsigned)grid);
  if (nw == 8 && !int8)
    hipLaunchKernelGGL((k_residue_persistent<8, false>), gr, dim3(64 * 8), 0, st, W);
  else if (nw == 4 && !int8)
    hipLaunchKernelGGL((k_residue_persistent<4, false>), gr, dim3(64 * 4), 0, st, W);
  else if (nw == 8)
    hipLaunchKernelGGL((k_residue_persistent<8, true>), gr, dim3(64 * 8), 0, st, W);
  else if (nw == 4)
    hipLaunchKernelGGL((k_residue_persistent<4, true>), gr, dim3(64 * 4), 0, st, W);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gemm_family(int fam, const Problem *P, const Group *G, hipStream_t st) {
  // grouped launches: the (unsplit) bound product only (a batch's residue
  // products run as one persistent launch)
  const bool grouped = G != nullptr;
  if (grouped && fam != kFamBgemm) return hipErrorInvalidValue;
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
  const dim3 gr((unsigned)blocks),
      blk(fam == kFamBgemm || fam == kFamBreduce ? 64 * NW_BOUND : 64 * NW_RES);
  switch (fam) {
    case kFamBgemm:
      if (grouped)
        hipLaunchKernelGGL((k_bound_gemm<true>), gr, blk, 0, st, p1, g1);
      else
        hipLaunchKernelGGL((k_bound_gemm<false>), gr, blk, 0, st, p1, g1);
      break;
    case kFamBreduce:
      hipLaunchKernelGGL(k_bound_reduce, gr, blk, 0, st, p1);
      break;
    case kFamGemmSq:
      hipLaunchKernelGGL((k_residue_gemm<0>), gr, blk, 0, st, p1);
      break;
    case kFamGemmKa:
      hipLaunchKernelGGL((k_residue_gemm<1>), gr, blk, 0, st, p1);
      break;
    case kFamGemmI8:
      hipLaunchKernelGGL((k_residue_gemm<2>), gr, blk, 0, st, p1);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace oz2
