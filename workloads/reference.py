"""Near-exact reference products for measuring the error of an emulated DGEMM.

Not part of the emulation: this computes op(A) op(B) for a sample of output
entries in double-double arithmetic, so that errors near 1e-16 |A||B| can be
measured.  Products are split exactly (Dekker's TwoProduct with Veltkamp
splitting) and summed by a pairwise tree of error-free TwoSums, keeping all
rounding errors in a low-order part.  The result's error is of order
log2(k) u^2 sum |a||b|, far below the quantities measured with it.
"""
from __future__ import annotations

import numpy as np

_SPLIT = 134217729.0  # 2^27 + 1


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    err = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, err


def _two_sum(a, b):
    s = a + b
    bb = s - a
    err = (a - (s - bb)) + (b - bb)
    return s, err


def dd_dot_rows(Ar: np.ndarray, Bc: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Double-double products of the rows of Ar (r x k) with the columns of
    Bc (k x c).  Returns (hi, lo) arrays of shape (r, c)."""
    Ar = np.asarray(Ar, dtype=np.float64)
    Bc = np.asarray(Bc, dtype=np.float64)
    r, k = Ar.shape
    c = Bc.shape[1]
    hi = np.zeros((r, c))
    lo = np.zeros((r, c))
    step = max(1, min(k, (1 << 22) // max(1, c)))
    for i in range(r):
        acc_hi = np.zeros(c)
        acc_lo = np.zeros(c)
        for h0 in range(0, k, step):
            a = Ar[i, h0:h0 + step][:, None]
            b = Bc[h0:h0 + step, :]
            p, e = _two_prod(np.broadcast_to(a, b.shape), b)
            low = e.sum(axis=0)
            x = p
            while x.shape[0] > 1:
                if x.shape[0] % 2:
                    x = np.concatenate([x, np.zeros((1, c))], axis=0)
                s, t = _two_sum(x[0::2], x[1::2])
                low = low + t.sum(axis=0)
                x = s
            s, t = _two_sum(acc_hi, x[0])
            acc_hi = s
            acc_lo = acc_lo + t + low
        s, t = _two_sum(acc_hi, acc_lo)
        hi[i], lo[i] = s, t
    return hi, lo


def normalised_error(C: np.ndarray, ref_hi: np.ndarray, ref_lo: np.ndarray,
                     absA: np.ndarray, absB: np.ndarray) -> float:
    """max_ij |C_ij - (AB)_ij| / (|A||B|)_ij over the sampled entries
    (entries with (|A||B|)_ij = 0 must match exactly and are skipped)."""
    den = absA @ absB
    diff = np.abs((C - ref_hi) - ref_lo)
    mask = den > 0
    if not np.any(mask):
        return 0.0
    return float(np.max(diff[mask] / den[mask]))
