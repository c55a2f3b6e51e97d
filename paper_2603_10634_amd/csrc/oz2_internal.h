// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ozaki2.h"

namespace oz2 {

constexpr int kMaxN = OZ2_MAX_MODULI;
constexpr int kLimbs = 8;        // 32-bit limbs for S = sum_l w_l u_l (< 2^256)
constexpr int kPad = 256;        // every dimension is padded to this multiple
constexpr int kChunkK = 1 << 15; // k handled by one residue-product launch

// Moduli and CRT constants for one N, built on the host (oz2_tables.cpp) and
// copied to device memory once per device and N.
struct Tables {
  int32_t N;                  // number of moduli
  int32_t M;                  // digit slices per operand: 2 per square, 3 otherwise
  int32_t limbs;              // 32-bit limbs of P
  int32_t reserved;
  int32_t p[kMaxN];           // moduli, hybrid order (Section III-D)
  int32_t s[kMaxN];           // digit radix: sqrt(p) for squares, 16 otherwise
  int32_t kind[kMaxN];        // 0 square (Section III-C), 1 Karatsuba (III-B)
  int32_t slice0[kMaxN];      // index of the modulus' first digit slice
  int32_t smag[kMaxN];        // ceil(2^16 / s): floor(v / s) = (v * smag) >> 16 for v <= 560
  int32_t kinit[kMaxN];       // Karatsuba: -16 / 15 mod p (symmetric), see the residue products
  int32_t pow2_32[kMaxN];     // 2^32 mod p
  int32_t pow2lo[kMaxN][64];  // 2^t mod p, t < 64
  int32_t pow2hi[kMaxN][4];   // 2^(64 t) mod p, t < 4
  float inv_p[kMaxN];         // 1/p, float
  double inv_pd[kMaxN];       // 1/p, double
  uint32_t w[kMaxN][kLimbs];  // CRT weights q_l P / p_l, little-endian limbs
  uint32_t P[kLimbs];         // product of the moduli
  uint32_t half[kLimbs];      // floor(P / 2)
  double P_d;                 // P rounded to double (estimate of quotients)
  double D;                   // largest double <= P - 1 (scale rule)
};

// Builds the tables for N moduli (host).  Returns false for an unsupported N.
bool build_tables(int N, Tables *t);

// Per-call geometry shared by the launchers.
struct Geometry {
  int64_t m, n, k;            // logical sizes
  int64_t mp, np, kp;         // padded sizes
  int N, M;
};

// Workspace views of one call.
struct Work {
  int32_t *shift;     // [mp + np] log2 mu_i, then log2 nu_j
  int32_t *E;         // [mp + np] ufp exponents
  int32_t *e;         // [mp + np] scale exponents
  uint64_t *amax;     // [mp + np] bits of max |x| per line
  uint32_t *rmax;     // [mp + np] FP32 bits of the bound product's line maxima
  uint32_t *flags;    // [mp + np]
  uint64_t *rfix;     // [mp + np] exact line maxima (FP64 bits) for fix-ups
  uint32_t *amb;      // [1 + mp + np] count, then the lines needing a fix-up
  uint8_t *Abar, *Bbar;
  uint8_t *Asl, *Bsl;
  int16_t *planes;
};

enum LineFlag : uint32_t { kNonFinite = 1u, kZeroLine = 2u, kFixup = 4u };

// Operand view: line r (row of op(A) or column of op(B)), k-index h at
// ptr[r * sr + h * sh].  Exactly one of sr, sh is 1.
struct Operand {
  const double *ptr;
  int64_t lines, k, sr, sh;
};

// ---- launchers (all asynchronous on `st`) ----
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st);
hipError_t launch_line_max(const Operand &op, uint64_t *amax, uint32_t *flags, hipStream_t st);
hipError_t launch_bound_operand(const Operand &op, int64_t lines_pad, int64_t kp,
                                const uint64_t *amax, int32_t *E, uint32_t *flags,
                                uint8_t *bar, hipStream_t st);
hipError_t launch_bound_gemm(const Geometry &g, const uint8_t *Abar, const uint8_t *Bbar,
                             uint32_t *rmaxA, uint32_t *rmaxB, hipStream_t st);
hipError_t launch_scale(const Geometry &g, const Tables *dt, const Work &w, hipStream_t st);
hipError_t launch_residues(const Operand &op, int64_t lines_pad, int64_t kp,
                           const int32_t *shift, const Tables *dt, int N, uint8_t *slices,
                           hipStream_t st);
hipError_t launch_residue_gemm(const Geometry &g, const Tables *dt, const uint8_t *Asl,
                               const uint8_t *Bsl, int16_t *planes, hipStream_t st);
hipError_t launch_crt(const Geometry &g, const Tables *dt, const Work &w, double alpha,
                      double beta, double *C, int64_t ldc, int limbs, hipStream_t st);
hipError_t launch_scal(int64_t m, int64_t n, double beta, double *C, int64_t ldc,
                       hipStream_t st);

}  // namespace oz2
