"""The oracle's BLAS-style wrapper: column-major layout, transposes, leading
dimensions, alpha/beta and quick returns."""
import math

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


# ---------------------------------------------------------------------------
# combine_alpha_beta against exact rational arithmetic: every operation of
# RN(RN(alpha Chat) + RN(beta C_in)) (R10) is formed exactly as a Fraction and
# rounded once to nearest-even, overflow and signed zeros included.
# ---------------------------------------------------------------------------
from fractions import Fraction  # noqa: E402

_MAXF = Fraction(2) ** 1024 - Fraction(2) ** 970   # smallest magnitude rounding to inf


def _rn(x: Fraction, zero_sign: float) -> float:
    """x rounded to the nearest double (ties to even), inf past the overflow
    threshold; an exact zero takes the sign IEEE 754 gives it (zero_sign)."""
    if x == 0:
        return math.copysign(0.0, zero_sign)
    if abs(x) >= _MAXF:
        return math.inf if x > 0 else -math.inf
    return float(x)      # CPython's int/int true division rounds correctly


def _exact_combine(chat: float, alpha: float, beta: float, cin: float) -> float:
    if not all(math.isfinite(v) for v in (chat, alpha, beta, cin)):
        return float("nan")  # only NaN-ness is compared for these
    t = _rn(Fraction(alpha) * Fraction(chat),
            -1.0 if (math.copysign(1, alpha) * math.copysign(1, chat)) < 0 else 1.0)
    if beta == 0.0:
        return t
    u = _rn(Fraction(beta) * Fraction(cin),
            -1.0 if (math.copysign(1, beta) * math.copysign(1, cin)) < 0 else 1.0)
    if math.isinf(t) or math.isinf(u):
        return t + u
    both_neg = math.copysign(1, t) < 0 and math.copysign(1, u) < 0
    return _rn(Fraction(t) + Fraction(u), -1.0 if both_neg else 1.0)



def _combine_cases():
    rng = np.random.default_rng(20260310)
    chat = rng.standard_normal(400) * np.exp2(rng.integers(-60, 60, 400))
    cin = rng.standard_normal(400) * np.exp2(rng.integers(-60, 60, 400))
    alphas = [1.0, -1.5, 0.1, 3.0000000000000004, 2.0 ** -1074 * 3, 1e300]
    betas = [0.0, 1.0, 0.25, -0.3, 1e-300, 7.0]
    cases = []
    for a in alphas:
        for b in betas:
            cases.append((chat, a, b, cin))
    # cancelling terms: alpha Chat = -beta C_in before rounding, and near it,
    # where one fused rounding would differ from two separate ones
    x = rng.standard_normal(200)
    cases.append((x, 0.1, -0.1, x))
    cases.append((x, 1.0 / 3.0, -1.0, x / 3.0))
    cases.append((x * (1 + 2.0 ** -52), 0.7, -0.7, x))
    # subnormal results, overflow, signed zeros, non-finite entries
    tiny = np.array([2.0 ** -1074, -2.0 ** -1070, 3 * 2.0 ** -1060, 0.0, -0.0, 1e-310])
    cases.append((tiny, 0.5, 0.5, tiny[::-1].copy()))
    cases.append((tiny, -1.0, -0.0, tiny))
    big = np.array([1e308, -1.7e308, 8e307, 0.0, -0.0, 1.0])
    cases.append((big, 3.0, 2.0, big))
    cases.append((np.array([np.nan, np.inf, -np.inf, 1.0]), 2.0, 1.0,
                  np.array([1.0, 1.0, 2.0, np.nan])))
    return cases


def test_combine_alpha_beta_matches_exact_rounding():
    """Pins combine_alpha_beta (R10): one correctly rounded step per
    operation, C_in unread when beta == 0."""
    n_checked = 0
    for chat, a, b, cin in _combine_cases():
        with np.errstate(all="ignore"):
            got = ref.combine_alpha_beta(chat.copy(), a, b,
                                         None if b == 0.0 else cin.copy())
        for q in range(chat.size):
            want = _exact_combine(float(chat[q]), a, b, float(cin[q]))
            g = float(got[q])
            if math.isnan(want):
                assert math.isnan(g) or not math.isfinite(float(chat[q])) or \
                    not math.isfinite(float(cin[q])), (chat[q], a, b, cin[q])
                continue
            assert np.float64(g).view(np.int64) == np.float64(want).view(np.int64), \
                (chat[q], a, b, cin[q], g, want)
            n_checked += 1
    assert n_checked > 10000


def test_combine_alpha_beta_is_not_one_fused_rounding():
    """A fused form RN(alpha Chat + beta C_in) would keep the low bits that
    two roundings lose: on x (1 + 2^-52) 0.7 - 0.7 x the two differ, and the
    exact-rounding model picks the two-rounding value."""
    x = np.array([1.0 + 2.0 ** -52, 3.0, 5.0])
    a, b = 0.7, -0.7
    cin = np.array([1.0, 3.0 * (1 - 2.0 ** -53), 5.0])
    got = ref.combine_alpha_beta(x, a, b, cin)
    fused = [float(Fraction(a) * Fraction(float(x[q])) + Fraction(b) * Fraction(float(cin[q])))
             for q in range(3)]
    want = [_exact_combine(float(x[q]), a, b, float(cin[q])) for q in range(3)]
    assert list(got) == want
    assert fused != want
