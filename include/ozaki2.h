/*
 * ozaki2.h - C ABI of the MI355X (gfx950) FP8 Ozaki-II DGEMM emulation.
 *
 * The library computes C <- alpha * op(A) op(B) + beta * C for FP64 matrices
 * by the Ozaki-II scheme with FP8 quantization, accurate or fast mode (Uchino,
 * Ozaki, Imamura, "Double-Precision Matrix Multiplication Emulation via
 * Ozaki-II Scheme with FP8 Quantization", arXiv 2603.10634):
 *   1. per-row / per-column power-of-two scaling of op(A), op(B) to integers
 *      A', B' (Section II eqs. def:A', def:B'), with the scale chosen from an
 *      FP8 bound product (accurate mode) or from Cauchy-Schwarz norms (fast
 *      mode, Section III-E);
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
 *   - Stream, workspace, timing, graph, autotune, mode and modulus-list
 *     settings are per host thread.
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
#define OZ2_ERR_SCRATCH      6  /* the problem exceeds the scratch buffer of
                                   ozaki2_dgemm_noalloc */

/* Largest number of moduli (the hybrid list keeps its six squares first for
 * N < 34, Section IV-B) and largest k handled in one call. */
#define OZ2_MAX_MODULI 33
#define OZ2_MAX_K      (1 << 18)

/* Scaling modes (ozaki2_set_mode). */
#define OZ2_MODE_ACCURATE 0
#define OZ2_MODE_FAST     1

/* Modulus lists (ozaki2_set_moduli_list). */
#define OZ2_MODULI_HYBRID    0
#define OZ2_MODULI_KARATSUBA 1
#define OZ2_MODULI_INT8      2

/*
 * ozaki2_dgemm - emulated DGEMM in the calling thread's mode (ozaki2_set_mode,
 * accurate by default).
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
 *                  the paper (P/2 > 2^110, about 55 effective bits) for the
 *                  default hybrid list (13 for the Karatsuba-only list).
 *
 * Quick returns: m == 0 or n == 0 does nothing; k == 0 or alpha == 0 sets
 * C <- beta*C (C <- 0, unread, when beta == 0).  A row of op(A) or column of
 * op(B) holding Inf or NaN yields NaN in every entry of C it contributes to.
 * k > OZ2_MAX_K returns OZ2_ERR_UNSUPPORTED, and so does m, n or k above
 * 2^40 or a workspace size that does not fit in size_t.
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
 * operands, one int16 residue plane per modulus and k part of the residue
 * products (see ozaki2_set_split) and per-line vectors, for the calling
 * thread's modulus list (ozaki2_set_moduli_list), m/n blocking
 * (ozaki2_set_blocking: slices and planes then cover one block) and split.
 * Returns 0 for invalid sizes, for m, n or k above 2^40 and when the size
 * does not fit in size_t.
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
 * operands, or their norms in fast mode), [1] bound product (empty in fast
 * mode), [2] scale exponents and fix-up, [3] residue
 * and digit pass, [4] residue products with modular reduction, [5] CRT and
 * inverse scaling.  `count` is the capacity of ms; returns the number of
 * entries written (6), or a negative value on error.
 */
int ozaki2_get_kernel_times(float *ms, int count);

/*
 * ozaki2_moduli - the moduli the library uses for N = num_moduli under the
 * calling thread's modulus list (ozaki2_set_moduli_list), written to
 * p[0..N-1], with kinds[l] = 0 for a square modulus (modular reduction split,
 * Section III-C), 1 for a Karatsuba modulus (Section III-B) and 2 for an INT8
 * modulus (Section II).  Either output may be NULL.  Returns 0 or -1 for an
 * invalid N.
 */
int ozaki2_moduli(int num_moduli, int32_t *p, int32_t *kinds);

/*
 * ozaki2_workspace_layout - byte offsets, inside the workspace, of the
 * intermediate buffers of a call of this shape, for inspection by tests:
 *   off[0] int32  [m_pad + n_pad]  log2 of mu_i / nu_j (shift applied to each line)
 *   off[1] int32  [m_pad + n_pad]  E with ufp(max|x|) = 2^E per line (0 for zero lines)
 *   off[2] int32  [m_pad + n_pad]  scale exponent e_i / f_j (log2(mu/mu'))
 *   off[3] uint8  [m_pad x k_pad]  Abar (E4M3 codes; accurate mode), k-blocked:
 *          element (row i, k h) at (h / 64) * 64 m_pad + 64 i + h % 64
 *   off[4] uint8  [n_pad x k_pad]  Bbar (column j of op(B) as line j; accurate mode),
 *          k-blocked with n_pad lines
 *   off[5] uint8  [M x m_pad x k_pad]  digit slices of A' (slice order below), each
 *          k-blocked like Abar (INT8 residues as two's-complement bytes)
 *   off[6] uint8  [M x n_pad x k_pad]  digit slices of B'
 *   off[7] int16  [N x n_pad x m_pad]  C'_l, entry (i, j) at l*n_pad*m_pad + j*m_pad + i;
 *          with k parts (ozaki2_set_split) one such copy per part, q*N*n_pad*m_pad
 *          apart, whose sum modulo p_l is C'_l (the last region of the layout)
 *   off[8] uint32 [m_pad + n_pad]  FP32 bits of the bound product's line maxima
 *          (accurate mode)
 *   off[9] uint32 [m_pad + n_pad]  line flags: 1 non-finite, 2 all zero, 4 exponent
 *          from an exact bound (fixed-up lines; every line in fast mode)
 *   off[10] uint32 [2 + m_pad + n_pad]  the lines whose scale exponent the FP8
 *          bound could not settle (recomputed exactly; accurate mode): their
 *          numbers among the rows of op(A) and the columns of op(B), then the
 *          rows' line indices from entry 2 up and the columns' from the last
 *          entry down
 * The layout, and so the workspace size, is the same in both modes.
 * Lines 0..m_pad-1 are rows of op(A), m_pad..m_pad+n_pad-1 columns of op(B).
 * Slices: modulus l contributes 2 (square) or 3 (Karatsuba) consecutive
 * slices, digit x1 first.  Also writes pads[0..2] = m_pad, n_pad, k_pad and
 * pads[3] = M when pads is not NULL.  `off` must hold 11 entries.  Returns the
 * number of offsets written (11), or a negative value for invalid sizes.
 * The layout is that of an unblocked call (m/n blocking off, or a problem
 * that fits one block).
 */
int ozaki2_workspace_layout(int64_t m, int64_t n, int64_t k, int num_moduli,
                            int64_t *off, int64_t *pads);

/*
 * ozaki2_workspace_parts - how an ozaki2_dgemm call of this shape splits k
 * under the calling thread's settings (ozaki2_set_split, ozaki2_set_blocking):
 * *parts = the k parts of the residue products, i.e. the copies of the
 * residue planes at off[7]; *bound_parts = the k parts of the bound product
 * (1: one pass; more: their FP32 part sums use the planes region first).
 * Either pointer may be NULL.  Returns 0, or -1 for invalid sizes (nothing
 * written).
 */
int ozaki2_workspace_parts(int64_t m, int64_t n, int64_t k, int num_moduli, int *parts,
                           int *bound_parts);

/*
 * ozaki2_dgemm_batched - `count` independent emulated DGEMMs
 *   C_q <- alpha_q op(A_q) op(B_q) + beta_q C_q,  q = 0 .. count-1,
 * of any (uneven) shapes, all with num_moduli moduli.  Every argument after
 * `count` except num_moduli is a HOST array of `count` entries with the
 * meaning ozaki2_dgemm gives it (the pointer arrays hold device pointers).
 * Each C_q is bit-identical to what ozaki2_dgemm returns for problem q.
 *
 * Execution: each kernel family of the method (line maxima, bound operands,
 * bound product, scale exponents, residues and digits, CRT) runs as ONE
 * grouped launch over all problems, whose blocks are mapped to (problem,
 * tile) through prefix sums of per-problem tile counts.  The residue products
 * of all problems, moduli, 256 x 256 output tiles and k parts run as ONE
 * persistent launch (one workgroup per CU) that hands out a work list,
 * longest item first, through an atomic counter.  Its configuration (the
 * tile program and the split-K limit, see ozaki2_set_schedule) is the
 * default, the autotuner's choice (ozaki2_set_autotune) or a forced one.
 * Split-K applies to problems with at most 4 output tiles per modulus and a
 * padded k of at least 512: their k range is cut into up to 4 parts whose
 * products go to separate copies of the residue planes, summed by the CRT.
 * Problems are packed into sub-batches whose workspaces fit the workspace at
 * once; sub-batches run one after another.
 * The per-batch descriptors are built on the host and uploaded once per
 * distinct argument list (the last 8 are cached per thread, with their
 * captured graphs, see ozaki2_set_graph).
 *
 * Workspace: problem q of a sub-batch uses the offsets of
 * ozaki2_workspace_layout, with one copy of the residue planes (2 N mp np
 * bytes, the last region), or 4 for a problem that split-K may apply to, at
 * the sum of the earlier problems' sizes (each its planes offset plus its
 * copies, rounded up to 256 bytes).  A caller workspace (ozaki2_set_workspace)
 * must hold the largest problem; the library-owned one grows to the whole
 * batch (ozaki2_workspace_bytes_batched), capped at 16 GiB.
 *
 * Returns 0; -i for invalid argument i in the order of this signature
 * (1 count < 0, 2 transA, 3 transB, 4 m, 5 n, 6 k, 7 alpha, 8 A, 9 lda,
 * 10 B, 11 ldb, 12 beta, 13 C, 14 ldc, 15 num_moduli; an array argument is
 * invalid when it is NULL or any entry is), nothing launched; or a positive
 * OZ2_ERR_* code.  Problems with m or n = 0 are skipped; k = 0 or alpha = 0
 * scales C by beta as in ozaki2_dgemm.  Timing (ozaki2_get_kernel_times)
 * covers batched calls that run as one sub-batch outside graph mode.
 */
int ozaki2_dgemm_batched(int count, const char *transA, const char *transB,
                         const int64_t *m, const int64_t *n, const int64_t *k,
                         const double *alpha, const double *const *A, const int64_t *lda,
                         const double *const *B, const int64_t *ldb, const double *beta,
                         double *const *C, const int64_t *ldc, int num_moduli);

/* ozaki2_workspace_bytes_batched - workspace for running the whole batch as
 * one sub-batch (the sum over problems with m, n, k > 0 of their sizes as
 * laid out for ozaki2_dgemm_batched); 0 for invalid sizes and when a
 * problem's size or the sum does not fit in size_t. */
size_t ozaki2_workspace_bytes_batched(int count, const int64_t *m, const int64_t *n,
                                      const int64_t *k, int num_moduli);

/*
 * ozaki2_set_graph - when on, the calling thread's ozaki2_dgemm and
 * ozaki2_dgemm_batched calls capture their launch sequence in a hipGraph the
 * first time an argument list (sizes, scalars, pointers, workspace) is seen,
 * on a private stream, and replay that graph on the set stream at every call
 * with the same arguments.  Captured graphs contain kernels only (buffers are
 * cleared by kernels, not memset nodes).  Replays need the workspace and the
 * matrices at the same addresses, which the argument match guarantees.
 * Timing is not recorded in graph mode.
 */
int ozaki2_set_graph(int on);

/*
 * ozaki2_set_autotune - when on, the first batched call of a new set of
 * problem shapes times the persistent residue products under each
 * configuration (see ozaki2_set_schedule) on the call's own data, keeps the
 * fastest for those shapes (process-wide) and then runs the call.  When the
 * environment variable OZ2_AUTOTUNE_CACHE names a file, choices are also
 * kept there per shape bucket (number of moduli, mode, modulus list and the
 * histogram of the problems over log2 of their output tiles per modulus and
 * log2 of their 256-blocks of k), read by later processes; a missing or
 * malformed file is ignored (default configuration, or tuning again).  Off
 * (default): the default configuration unless the shapes or their bucket
 * were tuned before.
 */
int ozaki2_set_autotune(int on);

/* ozaki2_get_schedule - residue-product configuration (0..5, see
 * ozaki2_set_schedule) of the calling thread's last batched call, or -1 if
 * there was none. */
int ozaki2_get_schedule(void);

/*
 * ozaki2_set_schedule - force the residue-product configuration of the
 * calling thread's subsequent batched calls, or -1 (default) to leave it to
 * the autotuner.  config / 3 is the tile program of the 256 x 256 output
 * tiles (0: eight waves of 128 x 64 outputs, two per SIMD; 1: four waves of
 * 128 x 128, one per SIMD); config % 3 the split-K limit (at most 1, 2 or 4
 * k parts).  Every configuration gives bit-identical results.  Returns 0, or
 * -1 for a value outside -1..5 (the setting is then unchanged).
 */
int ozaki2_set_schedule(int config);

/*
 * ozaki2_set_split - number of k parts of the residue products of the
 * calling thread's subsequent ozaki2_dgemm (and ozaki2_dgemm_noalloc) calls.
 * Each modulus kind's products are one launch of (256 x 256 output tiles) x
 * (moduli of the kind) x (k parts) workgroups, one per CU at a time; part q
 * covers the q-th of `parts` near-equal ranges of 256-blocks of k and writes
 * its own copy of the residue planes, which the CRT sums modulo p.  More
 * parts keep the CUs busy when the output has few tiles.  0 (default): the
 * library's rule, which minimises the launches' waves of workgroups per unit
 * of k over 1..8 parts of at least 2048 k each (1 part for large outputs).
 * 1..8: that many parts (at most one per 256-block of k).  Every setting
 * gives bit-identical results; the workspace grows by 2 N mp np bytes per
 * part beyond the first.  Returns 0, or -1 for a value outside 0..8 (the
 * setting is then unchanged).
 */
int ozaki2_set_split(int parts);

/*
 * ozaki2_set_mode - scaling mode of the calling thread's subsequent
 * ozaki2_dgemm and ozaki2_dgemm_batched calls (Section III-E).  Both modes
 * take mu_i = mu'_i 2^e_i, nu_j = nu'_j 2^f_j with e_i the largest integer
 * with 2^(2 e_i + 1) r_i <= P - 1 (f_j likewise from c_j), which gives
 * 2 sum_h |a'_ih||b'_hj| < P (condition (3)) since the entries of the bound
 * product Abar Bbar are at most sqrt(r_i c_j):
 *   OZ2_MODE_ACCURATE (default)  r_i, c_j are the row / column maxima of the
 *        FP8 bound product Abar Bbar: one more FP8 product (3N + 1 in all).
 *   OZ2_MODE_FAST  r_i, c_j are the squared Euclidean norms of the rows of
 *        Abar and columns of Bbar (the Cauchy-Schwarz bound), summed exactly:
 *        no bound product (3N products), but a looser scale, so wide-range
 *        inputs may need one more modulus for the same accuracy (the paper
 *        runs fast mode with 13 moduli against 12 in accurate mode).
 * Both modes are deterministic.  Returns 0, or -1 for an unknown mode (the
 * setting is then unchanged).
 */
int ozaki2_set_mode(int mode);

/* ozaki2_get_mode - the calling thread's scaling mode. */
int ozaki2_get_mode(void);

/*
 * ozaki2_set_moduli_list - modulus list of the calling thread's subsequent
 * calls (and of the workspace, layout and moduli queries):
 *   OZ2_MODULI_HYBRID (default)  Section III-D: the squares 1089, 1024, 961,
 *        841, 625, 529 first (modular-reduction split, Section III-C), then
 *        511, 509, 503, ... (Karatsuba split, s = 16).
 *   OZ2_MODULI_KARATSUBA  Section III-B: 513, 512, 511, 509, 505, ...
 *        (greedy pairwise coprime from 513), all with the Karatsuba split.
 *        Three FP8 products per modulus like the hybrid list, but a smaller
 *        P for the same N (P/2 > 2^115 needs N = 13 instead of 12), so about
 *        one more modulus for the same accuracy: an ablation of the hybrid
 *        list's saving.
 *   OZ2_MODULI_INT8  Section II, the INT8-based Ozaki-II scheme (the
 *        paper's baseline): 256, 255, 253, 251, 247, ... (greedy pairwise
 *        coprime from 256); each residue, in [-128, 127], is one INT8
 *        operand and each modulus costs ONE INT8 product (INT32
 *        accumulation, v_mfma_i32_32x32x32_i8).  P/2 > 2^109 needs N = 14.
 *        The scale exponents come from the same FP8 bound (or, in fast mode,
 *        the same norms) as the FP8 lists.
 * ozaki2_moduli reports kind 2 for INT8 moduli; the workspace holds one
 * slice per INT8 modulus (M = N).
 * Returns 0, or -1 for an unknown list (the setting is then unchanged).
 */
int ozaki2_set_moduli_list(int list);

/* ozaki2_get_moduli_list - the calling thread's modulus list. */
int ozaki2_get_moduli_list(void);

/*
 * ozaki2_set_blocking - m/n blocking of the calling thread's subsequent
 * ozaki2_dgemm calls (Section IV-C: blocking m and n, not k, reduces the
 * working memory while keeping the products long).  m_blk, n_blk: block
 * extents in outputs, multiples of 256, or 0 for no blocking in that
 * dimension.  A blocked call first derives the scale exponents of the WHOLE
 * problem (bound operands and bound product over all of op(A), op(B)), then
 * runs residues, residue products and CRT block by block into C; every block
 * therefore equals the unblocked result bit for bit.  The workspace holds the
 * per-line vectors and bound operands of the whole problem and the digit
 * slices and residue planes of one block (ozaki2_workspace_bytes follows the
 * setting): at 16384^3, N = 12 that is 23.1 GB unblocked against 5.0 GB with
 * 4096 x 4096 blocks.  op(A)'s residues are computed once per block row,
 * op(B)'s once per block column when there is a single block row and again
 * for every block otherwise.  Blocked calls record no stage timing.  Batched
 * calls are not blocked.  Returns 0, -1 (m_blk) or -2 (n_blk) for a negative
 * or unaligned extent (the setting is then unchanged).
 */
int ozaki2_set_blocking(int64_t m_blk, int64_t n_blk);

/* ozaki2_get_blocking - the calling thread's blocking (either pointer may be
 * NULL). */
int ozaki2_get_blocking(int64_t *m_blk, int64_t *n_blk);

/*
 * ozaki2_dgemm_noalloc - ozaki2_dgemm for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results (bit-identical C),
 * argument errors and quick returns as ozaki2_dgemm, in the calling thread's
 * mode, modulus list, m/n blocking and stream; it ignores the thread's
 * workspace, graph and timing settings.
 *
 * Its workspace is a fixed device buffer of OZ2_NOALLOC_SCRATCH_BYTES per
 * GPU, held by the library until the process ends.  A problem whose
 * workspace (ozaki2_workspace_bytes with the same blocking) exceeds it
 * returns OZ2_ERR_SCRATCH and launches nothing; m/n blocking
 * (ozaki2_set_blocking) lowers the need.  No call allocates: the first call
 * on a device only looks up the buffer's device address and copies the
 * moduli tables into a second fixed buffer (synchronously, so that first call
 * must not be made during stream capture).  Every call on a GPU uses the same
 * buffer, so calls that overlap on one GPU (other streams, other host
 * threads) race and must be ordered by the caller.
 */
#define OZ2_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int ozaki2_dgemm_noalloc(char transA, char transB, int64_t m, int64_t n, int64_t k,
                         double alpha, const double *A, int64_t lda,
                         const double *B, int64_t ldb, double beta,
                         double *C, int64_t ldc, int num_moduli);

/* ozaki2_release - free the calling thread's library-owned workspace, timing
 * events, cached batch plans and graphs. */
int ozaki2_release(void);

/* ozaki2_status_string - static description of a return code. */
const char *ozaki2_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* OZAKI2_H */
