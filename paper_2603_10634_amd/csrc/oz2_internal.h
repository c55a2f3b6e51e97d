// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ozaki2.h"

namespace oz2 {

constexpr int kMaxN = OZ2_MAX_MODULI;
constexpr int kLimbs = 11;       // 32-bit limbs for S = sum_l w_l u_l (P < 2^296 for N = 33)
constexpr int kPad = 256;        // every dimension is padded to this multiple
constexpr int kChunkK = 1 << 15; // longest k one residue-product accumulation covers
constexpr int kPowT = 192;       // 2^t mod p is tabulated for t < kPowT; the integer
                                 // a' = mant 2^t of an input never has t >= e + 8, and the
                                 // scale exponent e stays below 160 for N <= 33

// Moduli and CRT constants for one N, built on the host (oz2_tables.cpp) and
// copied to device memory once per device and N.
struct Tables {
  int32_t N;                  // number of moduli
  int32_t M;                  // digit slices per operand: 2 per square, 3 otherwise
  int32_t limbs;              // 32-bit limbs of P
  int32_t nsq;                // square moduli (they come first): min(N, 6) or 0
                              // (then the Karatsuba moduli, or the INT8 ones)
  int32_t nka;                // Karatsuba moduli
  int32_t reserved[3];
  int32_t p[kMaxN];           // moduli, hybrid order (Section III-D)
  int32_t s[kMaxN];           // digit radix: sqrt(p) for squares, 16 for Karatsuba
  int32_t kind[kMaxN];        // 0 square (Section III-C), 1 Karatsuba (III-B), 2 INT8 (II)
  int32_t slice0[kMaxN];      // index of the modulus' first slice (2, 3 or 1 slices)
  int32_t kfold[kMaxN][4];    // Karatsuba: multipliers of the two folds and the final
                              // reduction, and the slice (1 or 2) of the second pass;
                              // see the residue products
  float inv_p[kMaxN];         // 1/p, float
  double inv_pd[kMaxN];       // 1/p, double
  double inv_pair[kMaxN];     // 1/(p_l p_(l+1)), double (the residue pass reduces two
                              // consecutive moduli of one kind in one FP64 step)
  float inv_s[kMaxN];         // 1/s, float
  uint16_t pw[kMaxN][kPowT];  // 2^t mod p, t < kPowT
  uint32_t w[kMaxN][kLimbs];  // CRT weights q_l P / p_l, little-endian limbs
  double wd[kMaxN][kLimbs];   // the same limbs as doubles (exact)
  uint32_t P[kLimbs];         // product of the moduli
  uint32_t half[kLimbs];      // floor(P / 2)
  uint32_t top[kLimbs];       // P - 1 - floor(P / 2): the largest C'
  double Pdl[kLimbs];         // the limbs of P as doubles (exact)
  double crt_fast;            // |C'| estimates up to this are surely in range
  double P_d;                 // P rounded to double
  double inv_P_d;             // 1 / P_d (estimate of quotients S / P)
  double D;                   // largest double <= P - 1 (scale rule)
};

// Builds the tables for N moduli of list `list` (OZ2_MODULI_HYBRID,
// OZ2_MODULI_KARATSUBA or OZ2_MODULI_INT8) on the host.  Returns false for an
// unsupported N.
bool build_tables(int N, int list, Tables *t);

// Per-call geometry shared by the launchers.
struct Geometry {
  int64_t m, n, k;            // logical sizes
  int64_t mp, np, kp;         // padded sizes
  int N, M;
  int nsq;                    // square moduli (the first nsq of the list)
  int nka;                    // Karatsuba moduli (the next nka); the rest are INT8
  int list;                   // OZ2_MODULI_HYBRID, _KARATSUBA or _INT8
};

// Workspace views of one call.
struct Work {
  int32_t *shift;     // [mp + np] log2 mu_i, then log2 nu_j
  int32_t *E;         // [mp + np] ufp exponents
  int32_t *e;         // [mp + np] scale exponents
  uint64_t *amax;     // [mp + np] bits of max |x| per line
  uint32_t *rmax;     // [mp + np] FP32 bits of the bound product's line maxima
  uint32_t *flags;    // [mp + np]
  uint64_t *rfix;     // [mp + np] 2^18 x the exact line bound: bound-product maxima of
                      // fixed-up lines (accurate mode), squared norms (fast mode)
  uint32_t *amb;      // [2 + mp + np] the lines needing a fix-up: counts of rows of op(A)
                      // and of columns of op(B), then the rows' line indices from
                      // amb[2] up and the columns' from amb[1 + mp + np] down
  uint8_t *Abar, *Bbar;
  uint8_t *Asl, *Bsl;
  int16_t *planes;
  float *bpart;       // FP32 sums of the bound product's k parts (when split), laid
                      // over the planes, which are written only later
  uint32_t *zero;     // the buffers that start at zero (amax .. amb), contiguous
  int64_t zero_words;
  int64_t lineB;      // index of op(B)'s first line in the per-line vectors, counted
                      // from op(A)'s first line (mp, or a block's offset)
};

// kFixup: the line's exponent comes from the exact bound in rfix.
enum LineFlag : uint32_t { kNonFinite = 1u, kZeroLine = 2u, kFixup = 4u };

// Operand view: line r (row of op(A) or column of op(B)), k-index h at
// ptr[r * sr + h * sh].  Exactly one of sr, sh is 1.
struct Operand {
  const double *ptr;
  int64_t lines, k, sr, sh;
};

// Everything the kernels need about one emulated GEMM.
struct Problem {
  Operand A, B;        // op(A): lines are its m rows; op(B): its n columns
  Geometry g;
  Work w;
  const Tables *tab;   // device copy of the tables for g.N
  double alpha, beta;
  double *C;
  int64_t ldc;
  int32_t limbs;       // 32-bit limbs of P (host tables), selects the CRT kernel
  int32_t mode;        // OZ2_MODE_ACCURATE or OZ2_MODE_FAST (selects the launch sequence)
  int32_t parts;       // k parts of the residue products (split-K): the CRT sums this
                       // many copies of the residue planes, each N mp np entries apart
  int32_t bparts;      // k parts of the bound product (1: one pass with line maxima)
};

// One work item of the persistent residue-product launch: tile (tx, ty) of
// modulus l of problem `prob`, over k in [k0, k1) (multiples of 256, walked in
// chunks of at most kChunkK), written to copy `part` of the problem's residue
// planes.
struct ProductItem {
  int32_t prob;
  int16_t l, part;
  int32_t tx, ty;
  int32_t k0, k1;
};

// Work list of a persistent residue-product launch.  counters[0] hands out
// items, counters[1] counts finished workgroups; both are zero between
// launches (the last workgroup to finish clears them).
struct WorkList {
  const Problem *probs;
  const ProductItem *items;
  int64_t count;
  uint32_t *counters;
};

// Layout of the FP8 bound operands and of every digit slice ("k-blocked"):
// a buffer of R padded lines and kp padded k holds element (line r, k h) at
// byte (h / 64) (64 R) + 64 r + h % 64, i.e. blocks of 64 k, each block the
// 64-byte pieces of all R lines in line order.  One 64-k stage of a tile of
// consecutive lines is then one contiguous range of memory.
__host__ __device__ inline int64_t kblocked(int64_t r, int64_t h, int64_t R) {
  return (h >> 6) * (R << 6) + (r << 6) + (h & 63);
}

// Tile shapes of the kernels (the block grids below depend on them).
constexpr int kGemmTJ = 256;  // output columns j per tile
constexpr int kGemmTIW = 256; // output rows i per tile of the single-product kernels
                              // (Karatsuba products, bound product)
constexpr int kGemmBK = 64;   // k per pipeline stage
constexpr int kQL = 16;       // quantization passes: 16 lines x 128 k per block
constexpr int kQK = 128;

// Kernel families of the emulation, in launch order.  One launch of a family
// covers one problem or a whole group of problems (a batch).
enum Family : int {
  kFamFill = 0,   // zero the per-line accumulators
  kFamLmaxA,      // line maxima of op(A) / op(B)
  kFamLmaxB,
  kFamBarA,       // FP8 bound operands
  kFamBarB,
  kFamNormA,      // fast mode: squared norms of the bound operands' lines
  kFamNormB,
  kFamBgemm,      // FP8 bound product (line maxima, or per-part sums when split)
  kFamBreduce,    // split bound product: sum of the parts, line maxima
  kFamDecide,     // scale exponents from the FP8 bound
  kFamFixup,      // exact bound product for undecided lines
  kFamFinal,      // shifts
  kFamResA,       // residues and FP8 digits
  kFamResB,
  kFamGemmSq,     // residue products, square moduli (every k part in one launch)
  kFamGemmKa,     // residue products, Karatsuba moduli
  kFamGemmI8,     // residue products, INT8 moduli
  kFamCrt,        // CRT, inverse scaling, alpha / beta
  kNumFamilies
};

// k-split of the line-maxima pass.
struct LmaxShape {
  int64_t gx, splits, hchunk;
};

__host__ __device__ inline LmaxShape lmax_shape(const Operand &op) {
  LmaxShape s;
  if (op.sh == 1) {  // k contiguous: a wave per line and k chunk, ~2048 waves
    s.gx = (op.lines + 3) / 4;
    const int64_t splits = (2048 + s.gx - 1) / s.gx;
    int64_t h = (op.k + splits - 1) / splits;
    h = (h + 63) / 64 * 64;
    s.hchunk = h;
    s.splits = (op.k + h - 1) / h;
  } else {  // lines contiguous: a thread per line and k chunk
    s.gx = (op.lines + 255) / 256;
    int64_t splits = (4096 + s.gx - 1) / s.gx;
    if (splits > op.k) splits = op.k;
    s.hchunk = (op.k + splits - 1) / splits;
    s.splits = (op.k + s.hchunk - 1) / s.hchunk;
  }
  return s;
}

struct Dims {
  int64_t x, y, z;
};

// Block grid of family `fam` for one problem.  Blocks are numbered x fastest,
// then y, then z.
__host__ __device__ inline Dims family_dims(int fam, const Problem &P) {
  const Geometry &g = P.g;
  switch (fam) {
    case kFamFill: {
      int64_t b = (P.w.zero_words + 255) / 256;
      return {b < 64 ? b : 64, 1, 1};
    }
    case kFamLmaxA: {
      const LmaxShape s = lmax_shape(P.A);
      return {s.gx, s.splits, 1};
    }
    case kFamLmaxB: {
      const LmaxShape s = lmax_shape(P.B);
      return {s.gx, s.splits, 1};
    }
    case kFamBarA:
    case kFamNormA:
    case kFamResA:
      return {g.mp / kQL, g.kp / kQK, 1};
    case kFamBarB:
    case kFamNormB:
    case kFamResB:
      return {g.np / kQL, g.kp / kQK, 1};
    case kFamBgemm:
      return {g.mp / kGemmTIW, g.np / kGemmTJ, P.bparts};
    case kFamBreduce:  // (the wide tile's 16 MFMA blocks per wave) per tile
      return {16 * (g.mp / kGemmTIW) * (g.np / kGemmTJ), 1, P.bparts > 1 ? 1 : 0};
    case kFamDecide:
    case kFamFinal:
      return {(g.mp + g.np + 255) / 256, 1, 1};
    case kFamFixup: {  // one-wave workgroups walking the flagged lines' items
      int64_t b = (g.mp + g.np) / 8;
      return {b < 8 ? 8 : (b > 4096 ? 4096 : b), 1, 1};
    }
    case kFamGemmSq:
    case kFamGemmKa:
    case kFamGemmI8: {
      // z = part * (moduli of the kind) + modulus
      const int64_t nz = fam == kFamGemmSq ? g.nsq : (fam == kFamGemmKa ? g.nka : g.N - g.nsq - g.nka);
      return {g.mp / kGemmTIW, g.np / kGemmTJ, nz * P.parts};
    }
    case kFamCrt:
      return {(g.m + 63) / 64, (g.n + 3) / 4, 1};
    default:
      return {0, 1, 1};
  }
}

// k range [*k0, *k1) of part `part` of `parts` of the residue products: the
// kp / kPad blocks of 256 k dealt out as evenly as possible (no part is empty
// when parts <= kp / kPad).
__host__ __device__ inline void part_range(int64_t kp, int parts, int part, int64_t *k0,
                                           int64_t *k1) {
  const int64_t nb = kp / kPad;
  *k0 = (int64_t)part * nb / parts * kPad;
  *k1 = ((int64_t)part + 1) * nb / parts * kPad;
}

__host__ __device__ inline int64_t family_blocks(int fam, const Problem &P) {
  const Dims d = family_dims(fam, P);
  return d.x * d.y * d.z;
}

// A grouped launch: segment q covers problem order[q] and owns the blocks
// [start[q], start[q + 1]) of the launch (start[nseg] = total).  A launch of
// a single problem passes it by value instead and numbers its blocks from 0.
struct Group {
  const Problem *probs;
  const int32_t *order;
  const int64_t *start;
  const int32_t *seg;   // segment of every block (null: found by binary search in start)
  const Tables *tab;    // the device tables, the same for every problem of a batch: read
                        // through this kernel argument, they load with scalar loads
  int nseg;
  int64_t total;
};

// The device tables of the problem a block works on (see Group::tab).
template <bool GROUPED>
__host__ __device__ inline const Tables *tables_of(const Problem &P1, const Group &G) {
  return GROUPED ? G.tab : P1.tab;
}

#if defined(__HIPCC__)
// Segment holding block b: the last q with start[q] <= b (start is sorted;
// empty segments repeat a value).
__device__ __forceinline__ int find_segment(const Group &G, int64_t b) {
  int lo = 0, hi = G.nseg;  // start[lo] <= b < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (G.start[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The problem and local block number of block b: a single-problem launch
// passes its problem by value (P1), a grouped one a Group.
template <bool GROUPED>
__device__ __forceinline__ const Problem *locate(const Problem &P1, const Group &G, int64_t b,
                                                 int64_t &local) {
  if constexpr (GROUPED) {
    // one load from the per-block table where the plan has one (a binary
    // search costs a chain of dependent loads in every block)
    const int q = G.seg ? G.seg[b] : find_segment(G, b);
    local = b - G.start[q];
    return &G.probs[G.order[q]];
  } else {
    local = b;
    return &P1;
  }
}

// Local block coordinates of block `local` of a family grid.
__device__ __forceinline__ Dims decode_block(const Dims &d, int64_t local) {
  Dims c;
  c.x = local % d.x;
  const int64_t r = local / d.x;
  c.y = r % d.y;
  c.z = r / d.y;
  return c;
}
#endif

// ---- launchers (all asynchronous on `st`) ----
// Exactly one of P (a single problem, passed to the kernel by value) and G
// (a grouped launch over device-resident problems) is non-null.
// launch_gemm_family runs the residue products for a single problem only (a
// batch's run as launch_gemm_persistent).
hipError_t launch_quant_family(int fam, const Problem *P, const Group *G, hipStream_t st);
hipError_t launch_scale_family(int fam, const Problem *P, const Group *G, hipStream_t st);
hipError_t launch_gemm_family(int fam, const Problem *P, const Group *G, hipStream_t st);
// The persistent residue-product launch: `grid` workgroups of nw (8 or 4)
// waves take items of W in order until none is left; int8 selects the INT8
// arm's products (every item's modulus is then an INT8 one), else every
// item's modulus is a square or Karatsuba FP8 modulus.
hipError_t launch_gemm_persistent(int nw, bool int8, const WorkList &W, int64_t grid,
                                  hipStream_t st);
hipError_t launch_crt_family(const Problem *P, const Group *G, int limbs, int N, hipStream_t st);
// Device memory of the entry point that allocates nothing: a workspace and
// the device tables of every (modulus list, N), laid out [list][N - 1].
struct FixedResources {
  uint8_t *ws;
  size_t ws_bytes;
  const Tables *tables;
};

// ozaki2_dgemm's argument checks, quick returns and launch sequence (with the
// calling thread's stream, mode, modulus list and m/n blocking) on the
// workspace and tables that resources(dev) returns for the current device;
// never allocates, captures a graph or records timing events.  A problem
// whose workspace exceeds resources' returns OZ2_ERR_SCRATCH.
int dgemm_fixed(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                double *C, int64_t ldc, int num_moduli, FixedResources (*resources)(int dev));

// Host copy of the tables of N moduli of list `list` (false: unsupported).
bool host_tables_for(int N, int list, Tables *out);

hipError_t launch_scal(int64_t m, int64_t n, double beta, double *C, int64_t ldc,
                       hipStream_t st);

}  // namespace oz2
