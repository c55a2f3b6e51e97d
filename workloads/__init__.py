"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random matrices and lays them out in memory. It holds
none of the emulation's arithmetic, so both the CPU oracle and the HIP path
can be fed from it without sharing any part of the method.

Distribution (Numerical Results section, accuracy experiment): entries are
(rand - 0.5) * exp(randn * phi), where phi controls the spread of magnitudes,
plus a plain standard-normal variant. The paper draws them with cuRAND; here
numpy's PCG64 stands in, with the same distribution (uniform on [0, 1) instead
of (0, 1], which differs only at an endpoint of measure zero).
"""
from __future__ import annotations

import numpy as np

#: base seed; per-config seeds are derived as SEED_BASE + 100*config + 10*phi_index
SEED_BASE = 2603_10634


def config_seed(config: int, phi_index: int = 0) -> int:
    """Seed of op(A) for a workload; op(B) uses the next integer."""
    return SEED_BASE + 100 * config + 10 * phi_index


#: the spreads phi of each named workload, in the order that numbers their seeds
WORKLOAD_PHIS = {1: (0.5,), 2: (0.5, 2.0, 4.0), 3: (1.0,), 4: (1.0,), 5: (1.0, 6.0)}


def phi_seed(config: int, phi: float) -> int:
    """Seed of op(A) for spread phi of workload `config`: phi's position in
    that workload's list of spreads numbers it (0 for a spread not listed)."""
    phis = WORKLOAD_PHIS.get(config, ())
    idx = phis.index(float(phi)) if float(phi) in phis else 0
    return config_seed(config, idx)


def phi_matrix(rows: int, cols: int, phi: float, seed: int) -> np.ndarray:
    """(rows x cols) float64 with entries (U[0,1) - 0.5) * exp(phi * N(0,1)).

    Values are drawn row by row (C order) so that the same logical matrix
    comes out whatever memory layout it is later stored in.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((rows, cols))
    g = rng.standard_normal((rows, cols))
    return (u - 0.5) * np.exp(phi * g)


def normal_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """(rows x cols) float64 standard-normal entries ("Std. normal" inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((rows, cols))


def integer_matrix(rows: int, cols: int, bound: int, seed: int) -> np.ndarray:
    """(rows x cols) float64 holding integers drawn uniformly from [-bound, bound]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(-bound, bound + 1, size=(rows, cols)).astype(np.float64)


def cancellation_block(A: np.ndarray, B: np.ndarray, rows: int, cols: int,
                       eps: float, seed: int) -> np.ndarray:
    """Return a copy of op(A) whose first `rows` rows are orthogonal to the first
    `cols` columns of op(B), up to a relative perturbation `eps`.

    Used for the mixed-sign cancellation stress case: the exact products in that
    block are tiny compared with |A||B|.
    """
    A = A.copy()
    q, _ = np.linalg.qr(B[:, :cols])            # orthonormal basis of span(B[:, :cols])
    blk = A[:rows, :]
    blk = blk - (blk @ q) @ q.T                  # project rows onto the complement
    rng = np.random.Generator(np.random.PCG64(seed))
    pert = rng.standard_normal(blk.shape)
    norms = np.linalg.norm(blk, axis=1, keepdims=True)
    blk = blk + eps * norms * pert / np.sqrt(blk.shape[1])
    A[:rows, :] = blk
    return A


def to_colmajor(op: np.ndarray, trans: str, ld: int | None = None,
                fill: float = np.nan) -> tuple[np.ndarray, int]:
    """Store a logical operand op(X) as a flat column-major BLAS buffer.

    trans 'N': X = op(X), stored (ld x cols) column-major, ld >= rows.
    trans 'T'/'C': X = op(X)^T, stored (ld x rows) column-major, ld >= cols.
    Entries in the leading-dimension padding get `fill` (NaN by default, so a
    kernel that reads them shows it).  Returns (flat buffer, ld).
    """
    r, c = op.shape
    if trans in "Nn":
        ld = max(1, r) if ld is None else ld
        buf = np.full((c, ld), fill, dtype=np.float64)
        buf[:, :r] = op.T
    else:
        ld = max(1, c) if ld is None else ld
        buf = np.full((r, ld), fill, dtype=np.float64)
        buf[:, :c] = op
    return buf.reshape(-1), ld


def from_colmajor(buf: np.ndarray, rows: int, cols: int, ld: int) -> np.ndarray:
    """Read a (rows x cols) matrix out of a flat column-major buffer."""
    if rows == 0 or cols == 0:
        return np.zeros((rows, cols))
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    return np.lib.stride_tricks.as_strided(
        buf, shape=(rows, cols), strides=(8, 8 * ld)).copy()


def batch_shapes(count: int, lo: int, hi: int, seed: int) -> list[tuple[int, int, int]]:
    """`count` problem shapes (m, n, k), each dimension drawn independently and
    log-uniformly from [lo, hi] and rounded to an integer (the uneven batch of
    many small and mid-size products)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, 3)))
    x = np.clip(np.rint(x), lo, hi).astype(np.int64)
    return [tuple(int(v) for v in row) for row in x]
