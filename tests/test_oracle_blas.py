"""The oracle's BLAS-style wrapper: column-major layout, transposes, leading
dimensions, alpha/beta and quick returns."""
import numpy as np

from oracle import ozaki2_ref as ref
from workloads import phi_matrix, to_colmajor, from_colmajor


def _setup(m=13, n=9, k=21, seed=5):
    return phi_matrix(m, k, 1.0, seed), phi_matrix(k, n, 1.0, seed + 1)


def test_transposes_bit_identical():
    A, B = _setup()
    m, k = A.shape
    n = B.shape[1]
    want = ref.emulate(A, B, 12)
    for ta in "NT":
        for tb in "NT":
            Ab, lda = to_colmajor(A, ta, ld=(m + 3 if ta == "N" else k + 2))
            Bb, ldb = to_colmajor(B, tb, ld=(k + 1 if tb == "N" else n + 4))
            C = np.full(m * n, np.nan)
            out = ref.dgemm(ta, tb, m, n, k, 1.0, Ab, lda, Bb, ldb, 0.0, C, m, 12)
            assert np.array_equal(from_colmajor(out, m, n, m), want)


def test_alpha_beta():
    A, B = _setup()
    m, k = A.shape
    n = B.shape[1]
    Chat = ref.emulate(A, B, 12)
    Cin = phi_matrix(m, n, 1.0, 77)
    Cb, ldc = to_colmajor(Cin, "N", ld=m + 2, fill=7.0)
    Ab, lda = to_colmajor(A, "N")
    Bb, ldb = to_colmajor(B, "N")
    out = ref.dgemm("N", "N", m, n, k, -1.5, Ab, lda, Bb, ldb, 0.25, Cb, ldc, 12)
    assert np.array_equal(from_colmajor(out, m, n, ldc), -1.5 * Chat + 0.25 * Cin)
    # padding of C untouched
    assert np.all(out.reshape(n, ldc)[:, m:] == 7.0)


def test_quick_returns():
    A, B = _setup()
    m, k = A.shape
    n = B.shape[1]
    Ab, lda = to_colmajor(A, "N")
    Bb, ldb = to_colmajor(B, "N")
    Cin = phi_matrix(m, n, 1.0, 78)
    Cb, ldc = to_colmajor(Cin, "N")
    nanC = np.full(m * n, np.nan)
    # beta = 0: C is not read
    out = ref.dgemm("N", "N", m, n, 0, 1.0, Ab, lda, Bb, ldb, 0.0, nanC, m, 12)
    assert np.all(out == 0.0)
    out = ref.dgemm("N", "N", m, n, k, 0.0, Ab, lda, Bb, ldb, 2.0, Cb, ldc, 12)
    assert np.array_equal(from_colmajor(out, m, n, ldc), 2.0 * Cin)
    out = ref.dgemm("N", "N", m, n, k, 1.0, Ab, lda, Bb, ldb, 0.0, nanC, m, 12)
    assert not np.any(np.isnan(out))
    out = ref.dgemm("N", "N", 0, n, k, 1.0, Ab, lda, Bb, ldb, 0.0, Cb, ldc, 12)
    assert np.array_equal(out, Cb)


def test_row_major_identity():
    # row-major C = A B is column-major C^T = B^T A^T
    A, B = _setup(8, 6, 11)
    m, k = A.shape
    n = B.shape[1]
    Arm = A.reshape(-1)          # row-major A == column-major A^T (k x m, ld k)
    Brm = B.reshape(-1)          # column-major B^T (n x k, ld n)
    C = np.zeros(m * n)
    out = ref.dgemm("N", "N", n, m, k, 1.0, Brm, n, Arm, k, 0.0, C, n, 12)
    assert np.array_equal(out.reshape(m, n), ref.emulate(A, B, 12))
