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
//
// Layout: operand slices are K-contiguous (line r's k bytes at r * kp).  The
// MFMA "A" operand is fed from B's slices (rows j) and the "B" operand from
// A's slices (rows i), so the accumulator holds D[j][i] = (A'B')_ij and each
// lane owns consecutive i of C's column-major planes.
//
// Workgroup: 256 threads (4 waves), tile 256 (j) x 128 (i); each wave owns a
// 128 x 64 block as 4 x 2 MFMA tiles of 32 x 32.  K advances 64 per stage
// through an LDS ring of S stages filled by direct global-to-LDS loads
// (global_load_lds_dwordx4) issued S - 1 stages ahead, so HBM/L2 latency
// hides behind S - 1 stages of MFMAs; no VGPRs stage the operands.  LDS rows
// are 64 B with the four 16 B chunks of row r XOR-swizzled by
// ((r >> 1) ^ (r >> 3)) & 3, which keeps the fragment reads (ds_read_b128)
// free of bank conflicts.
#include "oz2_internal.h"

namespace oz2 {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int TJ = 256;                  // tile rows (j, from B's slices)
constexpr int TI = 128;                  // tile columns (i, from A's slices)
constexpr int BK = 64;                   // k per stage (one MFMA step)
constexpr int ROWB = 64;                 // LDS bytes per tile row
constexpr int BSZ = TJ * ROWB;           // bytes of one B-side slice tile
constexpr int ASZ = TI * ROWB;           // bytes of one A-side slice tile
constexpr int LDS_RING = 147456;         // 144 KB: 3 stages of 2 slices or 6 of 1

__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

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

enum Pattern { kSquare = 0, kKara1 = 1, kOne = 2 };

__device__ __forceinline__ v16f mfma_f8(v8i a, v8i b, v16f c) {
  // cbsz = blgp = 0 selects E4M3 for both operands; zero scale operands give
  // the unscaled instruction
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// Operand fragment of a 32-row sub-tile: lane l holds row (l % 32) and the 32
// k bytes of logical chunks 2 (l / 32) and 2 (l / 32) + 1.  Both MFMA operands
// are read with the same k assignment, so the dot products pair matching k.
__device__ __forceinline__ v8i lds_frag(const uint8_t *tile, int row0) {
  const int lane = threadIdx.x & 63;
  const int r = row0 + (lane & 31);
  const int g = lane >> 5;
  const int f = swz(r);
  const uint8_t *row = tile + r * ROWB;
  const v4i lo = *(const v4i *)(row + 16 * ((2 * g) ^ f));
  const v4i hi = *(const v4i *)(row + 16 * ((2 * g + 1) ^ f));
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Issue the direct-to-LDS loads of one stage (64 k) of NS slices per side into
// `buf`: NS x (4 + 2) instructions per wave, each filling 1 KB = 16 tile rows.
// Lane L of the instruction for rows 16q..16q+15 fetches row 16q + L/4, chunk
// (L & 3) ^ swz(row), which lands at physical chunk L & 3.
template <int NS>
__device__ __forceinline__ void stage_issue(const uint8_t *const *gB, const uint8_t *const *gA,
                                            int64_t kp, int64_t kofs, uint8_t *buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rsub = lane >> 2, pc = lane & 3;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = wave + 4 * u;
      const int r = 16 * q + rsub;
      const uint8_t *src = gB[s] + (int64_t)r * kp + kofs + 16 * (pc ^ swz(r));
      __builtin_amdgcn_global_load_lds(
          (const void *)src,
          (__attribute__((address_space(3))) void *)(buf + s * BSZ + q * 1024), 16, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = wave + 4 * u;
      const int r = 16 * q + rsub;
      const uint8_t *src = gA[s] + (int64_t)r * kp + kofs + 16 * (pc ^ swz(r));
      __builtin_amdgcn_global_load_lds(
          (const void *)src,
          (__attribute__((address_space(3))) void *)(buf + NS * BSZ + s * ASZ + q * 1024), 16,
          0, 0);
    }
  }
}

// Wait until this wave's loads of the current stage have landed while the
// `ahead` later stages (each NS x 6 loads per lane) may stay in flight.
template <int NS, int S>
__device__ __forceinline__ void wait_stage(int ahead) {
  constexpr int L = NS * 6;
  if (S > 5 && ahead >= 4) {
    wait_vm<(S > 5 ? 4 : 0) * L>();
  } else if (S > 4 && ahead == 3) {
    wait_vm<(S > 4 ? 3 : 0) * L>();
  } else if (S > 3 && ahead == 2) {
    wait_vm<(S > 3 ? 2 : 0) * L>();
  } else if (ahead == 1) {
    wait_vm<L>();
  } else {
    wait_vm<0>();
  }
}

// Accumulate over nk stages of 64 k.  gB[s] / gA[s] point at row j0 / i0 of
// the s-th B-side / A-side slice.  S-stage ring in `lds`; one barrier per
// stage both publishes the stage's loads and frees the buffer of the previous
// stage for the refill issued right after it.
template <int NS, int PAT>
__device__ __forceinline__ void kloop(const uint8_t *const *gB, const uint8_t *const *gA,
                                      int64_t kp, int64_t kbeg, int nk, uint8_t *lds,
                                      v16f (&acc0)[4][2], v16f (&acc1)[4][2]) {
  constexpr int STAGE = NS * (BSZ + ASZ);
  constexpr int S = NS == 2 ? 3 : 6;
  static_assert(S * STAGE <= LDS_RING, "LDS ring");
  const int wave = threadIdx.x >> 6;
  const int wj = wave >> 1, wi = wave & 1;
#pragma unroll
  for (int t = 0; t < S - 1; ++t)
    if (t < nk) stage_issue<NS>(gB, gA, kp, kbeg + (int64_t)t * BK, lds + t * STAGE);
  for (int kt = 0; kt < nk; ++kt) {
    const int ahead = (nk - 1 - kt) < (S - 2) ? (nk - 1 - kt) : (S - 2);
    wait_stage<NS, S>(ahead);
    __builtin_amdgcn_s_barrier();
    if (kt + S - 1 < nk)
      stage_issue<NS>(gB, gA, kp, kbeg + (int64_t)(kt + S - 1) * BK,
                      lds + ((kt + S - 1) % S) * STAGE);
    const uint8_t *base = lds + (kt % S) * STAGE;
    const uint8_t *lb0 = base;
    const uint8_t *la0 = base + NS * BSZ;
    if (PAT == kSquare) {
      // slices: 0 = digit x1, 1 = digit x2.  acc0 += A2 B2, acc1 += A1 B2 + A2 B1
      const uint8_t *lb1 = lb0 + BSZ, *la1 = la0 + ASZ;
      v8i fa1[2], fa2[2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        fa1[ti] = lds_frag(la0, wi * 64 + ti * 32);
        fa2[ti] = lds_frag(la1, wi * 64 + ti * 32);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        const v8i fb1 = lds_frag(lb0, wj * 128 + tj * 32);
        const v8i fb2 = lds_frag(lb1, wj * 128 + tj * 32);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
          acc0[tj][ti] = mfma_f8(fb2, fa2[ti], acc0[tj][ti]);
          acc1[tj][ti] = mfma_f8(fb2, fa1[ti], acc1[tj][ti]);
          acc1[tj][ti] = mfma_f8(fb1, fa2[ti], acc1[tj][ti]);
        }
      }
    } else if (PAT == kKara1) {
      // slices: 0 = digit x1, 1 = digit x3.  acc0 += A3 B3, acc1 += A1 B1
      const uint8_t *lb1 = lb0 + BSZ, *la1 = la0 + ASZ;
      v8i fa1[2], fa3[2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        fa1[ti] = lds_frag(la0, wi * 64 + ti * 32);
        fa3[ti] = lds_frag(la1, wi * 64 + ti * 32);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        const v8i fb1 = lds_frag(lb0, wj * 128 + tj * 32);
        const v8i fb3 = lds_frag(lb1, wj * 128 + tj * 32);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
          acc0[tj][ti] = mfma_f8(fb3, fa3[ti], acc0[tj][ti]);
          acc1[tj][ti] = mfma_f8(fb1, fa1[ti], acc1[tj][ti]);
        }
      }
    } else {
      v8i fa[2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) fa[ti] = lds_frag(la0, wi * 64 + ti * 32);
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        const v8i fb = lds_frag(lb0, wj * 128 + tj * 32);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) acc0[tj][ti] = mfma_f8(fb, fa[ti], acc0[tj][ti]);
      }
    }
    // this stage's LDS reads complete before any wave passes the next barrier
    wait_lgkm0();
  }
  // the ring is free for the next use only when every wave is done with it
  __builtin_amdgcn_s_barrier();
}

__device__ __forceinline__ void zero_acc(v16f (&a)[4][2]) {
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int v = 0; v < 16; ++v) a[tj][ti][v] = 0.0f;
}

// Symmetric remainder of |v| < 2^31 modulo p, in [-floor(p/2), ceil(p/2) - 1].
// The float quotient estimate is within 1 of the rounded quotient.
__device__ __forceinline__ int smod_i32(int v, int p, float inv_p) {
  const int lo = -(p >> 1), hi = p - 1 - (p >> 1);
  const int q = (int)rintf((float)v * inv_p);
  int r = v - q * p;
  if (r > hi) r -= p;
  if (r < lo) r += p;
  return r;
}

// KIND 0: square moduli (blockIdx.z = l), KIND 1: Karatsuba moduli
// (blockIdx.z = l - l0).
template <int KIND>
// (operand pointers carry no __restrict__: the prefetch fence in kloop must be
// able to order their loads)
__global__ __launch_bounds__(256, 1) void k_residue_gemm(const uint8_t *Asl, const uint8_t *Bsl,
                                                         int16_t *__restrict__ planes,
                                                         const Tables *__restrict__ tab,
                                                         int64_t mp, int64_t np, int64_t kp,
                                                         int64_t kbeg, int nk, int accumulate,
                                                         int l0) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[LDS_RING];
  const int l = l0 + blockIdx.z;
  const int64_t i0 = (int64_t)blockIdx.x * TI;
  const int64_t j0 = (int64_t)blockIdx.y * TJ;
  const int sl0 = tab->slice0[l];
  const int p = tab->p[l];
  const float inv = tab->inv_p[l];
  const int64_t sA = mp * kp, sB = np * kp;
  const uint8_t *A0 = Asl + (int64_t)sl0 * sA + i0 * kp;
  const uint8_t *B0 = Bsl + (int64_t)sl0 * sB + j0 * kp;

  v16f acc0[4][2], acc1[4][2];
  zero_acc(acc0);
  zero_acc(acc1);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wj = wave >> 1, wi = wave & 1;
  int16_t *out = planes + (int64_t)l * np * mp;
  // accumulator element (tj, ti, v) of this lane is entry (i, j) of C'_l
  auto store = [&](int tj, int ti, int v, int r) {
    const int64_t i = i0 + wi * 64 + ti * 32 + (lane & 31);
    const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
    int16_t *dst = out + j * mp + i;
    if (accumulate) r = smod_i32(r + (int)*dst, p, inv);
    *dst = (int16_t)r;
  };

  if (KIND == 0) {
    const uint8_t *gB[2] = {B0, B0 + sB};
    const uint8_t *gA[2] = {A0, A0 + sA};
    kloop<2, kSquare>(gB, gA, kp, kbeg, nk, lds, acc0, acc1);
    const int s = tab->s[l];
    // eq. 3matmult-notKaratsuba: s (A1 B2 + A2 B1) + A2 B2 (mod s^2)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          store(tj, ti, v, smod_i32(s * (int)acc1[tj][ti][v] + (int)acc0[tj][ti][v], p, inv));
  } else {
    {
      const uint8_t *gB[2] = {B0, B0 + 2 * sB};
      const uint8_t *gA[2] = {A0, A0 + 2 * sA};
      kloop<2, kKara1>(gB, gA, kp, kbeg, nk, lds, acc0, acc1);
    }
    // eq. C'-Karatsuba with s = 16: 240 C1 - 15 C2 + 16 C3 = 16 t - 15 C2 with
    // t = 15 C1 + C3.  Modulo p this is -15 (C2 + t'), t' = kinit t: the
    // second pass starts its accumulator at t' (|t'| < 256, so the sum stays
    // an exact FP32 integer) and adds C2 on top.
    const int kinit = tab->kinit[l];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int t = smod_i32(15 * (int)acc1[tj][ti][v] + (int)acc0[tj][ti][v], p, inv);
          acc0[tj][ti][v] = (float)smod_i32(kinit * t, p, inv);
        }
    {
      const uint8_t *gB[1] = {B0 + sB};
      const uint8_t *gA[1] = {A0 + sA};
      kloop<1, kOne>(gB, gA, kp, kbeg, nk, lds, acc0, acc1);
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          store(tj, ti, v, smod_i32(-15 * (int)acc0[tj][ti][v], p, inv));
  }
}

__global__ __launch_bounds__(256, 1) void k_bound_gemm(const uint8_t *Abar, const uint8_t *Bbar,
                                                       int64_t kp, int nk,
                                                       uint32_t *__restrict__ rmaxA,
                                                       uint32_t *__restrict__ rmaxB) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[LDS_RING];
  const int64_t i0 = (int64_t)blockIdx.x * TI;
  const int64_t j0 = (int64_t)blockIdx.y * TJ;
  v16f acc0[4][2], acc1[4][2];
  zero_acc(acc0);
  const uint8_t *gB[1] = {Bbar + j0 * kp};
  const uint8_t *gA[1] = {Abar + i0 * kp};
  kloop<1, kOne>(gB, gA, kp, 0, nk, lds, acc0, acc1);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wj = wave >> 1, wi = wave & 1;
  // maxima over j of each column i (row maxima of Abar Bbar, for mu)
#pragma unroll
  for (int ti = 0; ti < 2; ++ti) {
    float m = 0.0f;
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int v = 0; v < 16; ++v) m = fmaxf(m, acc0[tj][ti][v]);
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    if (lane < 32)
      atomicMax(&rmaxA[i0 + wi * 64 + ti * 32 + lane], __float_as_uint(m));
  }
  // maxima over i of each row j (column maxima of Abar Bbar, for nu)
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float m = fmaxf(acc0[tj][0][v], acc0[tj][1][v]);
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
      if ((lane & 31) == 0) {
        const int64_t j = j0 + wj * 128 + tj * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        atomicMax(&rmaxB[j], __float_as_uint(m));
      }
    }
}

}  // namespace

hipError_t launch_bound_gemm(const Geometry &g, const uint8_t *Abar, const uint8_t *Bbar,
                             uint32_t *rmaxA, uint32_t *rmaxB, hipStream_t st) {
  dim3 grid((unsigned)(g.mp / TI), (unsigned)(g.np / TJ));
  hipLaunchKernelGGL(k_bound_gemm, grid, dim3(256), 0, st, Abar, Bbar, g.kp, (int)(g.kp / BK),
                     rmaxA, rmaxB);
  return hipGetLastError();
}

hipError_t launch_residue_gemm(const Geometry &g, const Tables *dt, const uint8_t *Asl,
                               const uint8_t *Bsl, int16_t *planes, hipStream_t st) {
  // the hybrid list puts its squares first: moduli 0..nsq-1 are squares
  const int nsq = g.N < 6 ? g.N : 6;
  for (int64_t k0 = 0; k0 < g.kp; k0 += kChunkK) {
    const int64_t len = g.kp - k0 < kChunkK ? g.kp - k0 : kChunkK;
    const int acc = k0 > 0 ? 1 : 0;
    hipLaunchKernelGGL(k_residue_gemm<0>, dim3((unsigned)(g.mp / TI), (unsigned)(g.np / TJ), nsq),
                       dim3(256), 0, st, Asl, Bsl, planes, dt, g.mp, g.np, g.kp, k0,
                       (int)(len / BK), acc, 0);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (g.N > nsq) {
      hipLaunchKernelGGL(k_residue_gemm<1>,
                         dim3((unsigned)(g.mp / TI), (unsigned)(g.np / TJ), g.N - nsq),
                         dim3(256), 0, st, Asl, Bsl, planes, dt, g.mp, g.np, g.kp, k0,
                         (int)(len / BK), acc, nsq);
      err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
  }
  return hipSuccess;
}

}  // namespace oz2
