"""Closed-form models printed in the paper (Section IV-B, IV-C).

Test infrastructure only.  These are reporting aids: the working-memory
formulas of eq. W8i / W8f and the analytic time models, written as printed.
"""
from __future__ import annotations


def num_slices(N: int) -> int:
    """M_N, the number of FP8 slices per operand (eq. M): 2N while every
    modulus is a square (N <= 6), else 3N - 6 (six squares, the rest Karatsuba)."""
    return 2 * N if N <= 6 else 3 * N - 6


def workspace_int8(m: int, n: int, k: int, N: int) -> int:
    """eq. W8i: (mk + kn + 5mn) N + 2(m + n) bytes."""
    return (m * k + k * n + 5 * m * n) * N + 2 * (m + n)


def workspace_fp8(m: int, n: int, k: int, N: int) -> int:
    """eq. W8f: (mk + kn + 4mn) M_N + 2 N mn + 2(m + n) bytes."""
    return (m * k + k * n + 4 * m * n) * num_slices(N) + 2 * N * m * n + 2 * (m + n)


def time_i8_acc(m, n, k, N, c, ops, b):
    """T_i8acc (Section IV-B)."""
    return (2 * m * n * k * (N + 1) / ops + (20 + 6 * N + 2 * c) * m * n / b
            + (((17 + N + c) * k + 4) * (m + n) + 2 * k * m + 2 * n) / b)


def time_i8_fast(m, n, k, N, c, ops, b):
    """T_i8fast (Section IV-B)."""
    return (2 * m * n * k * N / ops + (12 + 6 * N + 2 * c) * m * n / b
            + ((16 + N + c) * k + 2) * (m + n) / b)


def time_f8_acc(m, n, k, N, c, ops, b, gemms=None):
    """T_f8acc (Section IV-B).  As printed the GEMM term counts N + 1 products;
    `gemms` overrides that count (3N + 1 is the number the method performs)."""
    g = (N + 1) if gemms is None else gemms
    M = num_slices(N)
    return (2 * m * n * k * g / ops + (20 + 2 * c + 4 * N + 4 * M) * m * n / b
            + (((17 + M + c) * k + 4) * (m + n) + 2 * k * m + 2 * n) / b)


def time_f8_fast(m, n, k, N, c, ops, b, gemms=None):
    """T_f8fast (Section IV-B), with the same `gemms` override."""
    g = N if gemms is None else gemms
    M = num_slices(N)
    return (2 * m * n * k * g / ops + (12 + 2 * c + 4 * N + 4 * M) * m * n / b
            + ((16 + M + c) * k + 2) * (m + n) / b)
