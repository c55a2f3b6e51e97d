/*
 * ozaki2.h - C ABI of the MI355X (gfx950) FP8 Ozaki-II DGEMM emulation.
 *
 * The library computes C <- alpha * op(A) op(B) + beta * C for FP64 matrices
 * by the Ozaki-II scheme with FP8 quantization, accurate mode (Uchino, Ozaki,
 * Imamura, "Double-Precision Matrix Multiplication Emulation via Ozaki-II
 * Scheme with FP8 Quantization", arXiv 2603.10634):
 *   1. per-row / per-column power-of-two scaling of op(A), op(B) to integers
 *      A', B' (Section II eqs. def:A', def:B'), with the scale chosen from an
 *      FP8 bound product (Section III-E);
 *   2. residues of A', B' modulo the hybrid moduli 1089, 1024, 961, 841, 625,
 *      529, 511, 509, ... (Section III-D), split into FP8 E4M3 digits;
 *   3. three exact FP8 products per modulus on e4m3 MFMA with FP32
 *      accumulation (Sections III-B, III-C), reduced modulo p;
 *   4. Chinese-remainder reconstruction (eq. CRT_finalreduction) and inverse
 *      scaling back to FP64 (eq. inversescaling), rounded once to nearest.
 *
 * Conventions for every entry point:
 *   - Matrices are column-major (BLAS).  A row-major product C = A B is the
 *     column-major product C^T = B^T A^T, i.e.
 *       ozaki2_dgemm('N','N', n, m, k, alpha, B, n, A, k, beta, C, n, N).
 *   - A, B, C and workspace pointers are DEVICE pointers owned by the caller;
 *     sizes, alpha and beta are host values.  The library keeps no pointer to
 *     A, B or C after a call returns.
 *   - Work is enqueued on the stream set by ozaki2_set_stream (default: the
 *     null stream) and runs asynchronously; inputs must stay valid and
 *     unmodified until the stream reaches the end of the call.
 *   - Stream, workspace and timing settings are per host thread.
 *   - Results are deterministic: the same inputs give bit-identical C on every
 *     call and for all four transA/transB storage combinations.
 *
 * Return values: 0 on success; -i when argument i (1-based, BLAS order) is
 * invalid, in which case nothing is launched; a positive OZ2_ERR_* code for
 * run-time failures.
 */
#ifndef OZAKI2_H
#define OZAKI2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OZ2_SUCCESS          0
#define OZ2_ERR_HIP          1  /* a HIP runtime call or kernel launch failed */
#define OZ2_ERR_ALLOC        2  /* the library could not allocate its workspace */
#define OZ2_ERR_WORKSPACE    3  /* the caller's workspace is smaller than required */
#define OZ2_ERR_UNSUPPORTED  4  /* valid arguments outside what is built (see below) */
#define OZ2_ERR_NO_DEVICE    5  /* no gfx950 device is current */

/* Largest number of moduli (the hybrid list keeps its six squares first for
 * N < 34, Section IV-B) and largest k handled in one call. */
#define OZ2_MAX_MODULI 20
#define OZ2_MAX_K      (1 << 18)

/*
 * ozaki2_dgemm - emulated DGEMM, accurate mode.
 *
 *  transA, transB  'N'/'n' (op(X) = X) or 'T'/'t'/'C'/'c' (op(X) = X^T).
 *  m, n, k         op(A) is m x k, op(B) is k x n, C is m x n; each >= 0.
 *  alpha, beta     host scalars.  C = RN(alpha*Chat) when beta == 0 (C is not
 *                  read), else RN(RN(alpha*Chat) + RN(beta*C)); Chat is the
 *                  emulated product, rounded once to nearest-even.
 *  A, lda          device pointer; lda >= max(1, m) for 'N', >= max(1, k) else.
 *  B, ldb          device pointer; ldb >= max(1, k) for 'N', >= max(1, n) else.
 *  C, ldc          device pointer; ldc >= max(1, m).
 *  num_moduli      N in [1, OZ2_MAX_MODULI]; 12 is the full-accuracy count of
 *                  the paper (P/2 > 2^110, about 55 effective bits).
 *
 * Quick returns: m == 0 or n == 0 does nothing; k == 0 or alpha == 0 sets
 * C <- beta*C (C <- 0, unread, when beta == 0).  A row of op(A) or column of
 * op(B) holding Inf or NaN yields NaN in every entry of C it contributes to.
 * k > OZ2_MAX_K returns OZ2_ERR_UNSUPPORTED.
 * Argument indices for -i: 1 transA, 2 transB, 3 m, 4 n, 5 k, 8 lda, 10 ldb,
 * 13 ldc, 14 num_moduli.
 */
int ozaki2_dgemm(char transA, char transB, int64_t m, int64_t n, int64_t k,
                 double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta,
                 double *C, int64_t ldc, int num_moduli);

/*
 * ozaki2_workspace_bytes - device workspace one ozaki2_dgemm call of this
 * shape needs (every dimension padded to a multiple of 256, as in the paper's
 * Section IV-C): the FP8 bound operands, the FP8 digit slices of both
 * operands, one int16 residue plane per modulus and per-line vectors.
 * Returns 0 for invalid sizes.
 */
size_t ozaki2_workspace_bytes(int64_t m, int64_t n, int64_t k, int num_moduli);

/*
 * ozaki2_set_stream - stream (hipStream_t passed as void*) on which the calling
 * thread's subsequent calls enqueue their work; NULL selects the null stream.
 */
int ozaki2_set_stream(void *stream);

/*
 * ozaki2_set_workspace - use caller-owned device memory [ptr, ptr + bytes) as
 * the workspace of the calling thread's subsequent calls (256-byte aligned).
 * A call whose need exceeds `bytes` fails with OZ2_ERR_WORKSPACE.  Passing
 * NULL returns to the library-owned workspace, which grows on demand and is
 * released by ozaki2_release().
 */
int ozaki2_set_workspace(void *ptr, size_t bytes);

/*
 * ozaki2_set_timing - when on (nonzero), each call records HIP events between
 * its stages on the call's stream; ozaki2_get_stage_times reads them.
 */
int ozaki2_set_timing(int on);

/*
 * ozaki2_get_stage_times - milliseconds of the calling thread's last timed
 * call, split as in the paper's time breakdown (Section V-C):
 *   ms[0] quant   (scaling passes, bound operands, residues and FP8 digits)
 *   ms[1] gemms   (the FP8 bound product and the residue products)
 *   ms[2] requant (0: the modular reduction runs in the residue-product epilogue)
 *   ms[3] dequant (CRT reconstruction, inverse scaling, alpha/beta)
 *   ms[4] others  (scale-exponent derivation and its exact fix-up)
 * Synchronizes on the recorded events.  Returns OZ2_ERR_UNSUPPORTED when no
 * timed call has run on this thread.
 */
int ozaki2_get_stage_times(float ms[5]);

/*
 * ozaki2_get_kernel_times - milliseconds of each kernel group of the last
 * timed call, in launch order: [0] scaling pass 1 (maxima and bound
 * operands), [1] bound product, [2] scale exponents and fix-up, [3] residue
 * and digit pass, [4] residue products with modular reduction, [5] CRT and
 * inverse scaling.  `count` is the capacity of ms; returns the number of
 * entries written (6), or a negative value on error.
 */
int ozaki2_get_kernel_times(float *ms, int count);

/*
 * ozaki2_moduli - the moduli the library uses for N = num_moduli, written to
 * p[0..N-1], with kinds[l] = 0 for a square modulus (modular reduction split,
 * Section III-C) and 1 for a Karatsuba modulus (Section III-B).  Either output
 * may be NULL.  Returns 0 or -1 for an invalid N.
 */
int ozaki2_moduli(int num_moduli, int32_t *p, int32_t *kinds);

/*
 * ozaki2_workspace_layout - byte offsets, inside the workspace, of the
 * intermediate buffers of a call of this shape, for inspection by tests:
 *   off[0] int32  [m_pad + n_pad]  log2 of mu_i / nu_j (shift applied to each line)
 *   off[1] int32  [m_pad + n_pad]  E with ufp(max|x|) = 2^E per line (0 for zero lines)
 *   off[2] int32  [m_pad + n_pad]  scale exponent e_i / f_j (log2(mu/mu'))
 *   off[3] uint8  [m_pad x k_pad]  Abar, row i at i*k_pad (E4M3 codes)
 *   off[4] uint8  [n_pad x k_pad]  Bbar, column j of op(B) at j*k_pad
 *   off[5] uint8  [M x m_pad x k_pad]  digit slices of A' (slice order below)
 *   off[6] uint8  [M x n_pad x k_pad]  digit slices of B'
 *   off[7] int16  [N x n_pad x m_pad]  C'_l, entry (i, j) at l*n_pad*m_pad + j*m_pad + i
 *   off[8] uint32 [m_pad + n_pad]  FP32 bits of the bound product's line maxima
 *   off[9] uint32 [m_pad + n_pad]  line flags: 1 non-finite, 2 all zero, 4 exact fix-up
 *   off[10] uint32 [1 + m_pad + n_pad]  number of lines whose scale exponent
 *          the FP8 bound could not settle (recomputed exactly), then their indices
 * Lines 0..m_pad-1 are rows of op(A), m_pad..m_pad+n_pad-1 columns of op(B).
 * Slices: modulus l contributes 2 (square) or 3 (Karatsuba) consecutive
 * slices, digit x1 first.  Also writes pads[0..2] = m_pad, n_pad, k_pad and
 * pads[3] = M when pads is not NULL.  `off` must hold 11 entries.  Returns the
 * number of offsets written (11), or a negative value for invalid sizes.
 */
int ozaki2_workspace_layout(int64_t m, int64_t n, int64_t k, int num_moduli,
                            int64_t *off, int64_t *pads);

/* ozaki2_release - free the calling thread's library-owned workspace and
 * timing events. */
int ozaki2_release(void);

/* ozaki2_status_string - static description of a return code. */
const char *ozaki2_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* OZAKI2_H */
