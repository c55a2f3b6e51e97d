"""Pins for the oracle's scaling, residue products, CRT and final result.

Each check compares against something the oracle does not compute itself:
brute force with Python integers or exact rationals, the paper's condition (3)
evaluated exactly, closed-form special cases (integer inputs), analytic error
bounds, and symmetry invariants.  The check functions are reused by
test_oracle_mutations.py, which plants plausible mistakes in the oracle and
confirms that at least one check catches each."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import ozaki2_ref as ref
from workloads import phi_matrix, integer_matrix
from workloads.reference import dd_dot_rows, normalised_error


def _small_problem(m, n, k, phi, seed):
    A = phi_matrix(m, k, phi, seed)
    B = phi_matrix(k, n, phi, seed + 1)
    return A, B


# ---- check functions (return None on success, raise AssertionError) -------

def check_scale_exponent_brute(P, r18_values):
    for r18 in r18_values:
        e = ref.scale_exponent(r18, P)
        if r18 == 0:
            assert e == 0
            continue
        r = Fraction(int(r18), 2 ** 18)
        assert r * Fraction(2) ** (2 * e + 1) <= P - 1
        assert r * Fraction(2) ** (2 * e + 3) > P - 1


def check_condition3(A, B, N, mode="accurate", moduli_set="hybrid"):
    """2 sum_h |a'_ih||b'_hj| < P for all i, j, in exact integers (eq. condition)."""
    _, st = ref.emulate(A, B, N, keep_stages=True, mode=mode, moduli_set=moduli_set)
    Ai = [[int(x) for x in row] for row in st["Aint"]]
    Bi = [[int(x) for x in row] for row in st["Bint"]]
    m, k = len(Ai), len(Bi)
    n = len(Bi[0]) if k else 0
    for i in range(m):
        for j in range(n):
            s = sum(abs(Ai[i][h]) * abs(Bi[h][j]) for h in range(k))
            assert 2 * s < st["P"]


def check_bound_dominates(A, B, N):
    """mu'|A| nu'-products are bounded by the bound product (Section III-E)."""
    _, st = ref.emulate(A, B, N, keep_stages=True)
    m, k = A.shape
    n = B.shape[1]
    for i in range(m):
        for j in range(n):
            exact = sum(Fraction(abs(float(A[i, h]))) * Fraction(abs(float(B[h, j])))
                        for h in range(k))
            exact *= Fraction(2) ** (7 - int(st["EA"][i])) * Fraction(2) ** (7 - int(st["EB"][j]))
            bound = sum(Fraction(float(st["Abar"][i, h])) * Fraction(float(st["Bbar"][h, j]))
                        for h in range(k))
            assert exact <= bound
            assert bound * 2 ** 18 <= st["r18"][i] and bound * 2 ** 18 <= st["c18"][j]


def check_residue_products(A, B, N, moduli_set="hybrid"):
    """Per modulus: the direct product and the three-digit-product route both
    equal (A'B' mod p) computed with Python integers (eqs. CRTmatmul,
    Karatsuba, 3matmult-notKaratsuba)."""
    _, st = ref.emulate(A, B, N, keep_stages=True, moduli_set=moduli_set)
    Ai = [[int(x) for x in row] for row in st["Aint"]]
    Bi = [[int(x) for x in row] for row in st["Bint"]]
    m, k = len(Ai), len(Bi)
    n = len(Bi[0])
    exact = [[sum(Ai[i][h] * Bi[h][j] for h in range(k)) for j in range(n)] for i in range(m)]
    for pm, plane in zip(st["per_modulus"], st["planes"]):
        p = pm["p"]
        want = np.array([[ref.smod(exact[i][j], p) for j in range(n)] for i in range(m)])
        assert np.array_equal(plane, want)
        via = ref.residue_product_fp8(pm["dA"], pm["dB"], p, pm["kind"], pm["s"])
        assert np.array_equal(via, want)
        # the residues themselves: smod of the exact integers
        assert all(pm["uA"][i][h] == ref.smod(Ai[i][h], p) for i in range(m) for h in range(k))


def check_crt_is_exact_product(A, B, N, moduli_set="hybrid"):
    """C' equals the exact integer product A'B' (Section II: exact products)."""
    _, st = ref.emulate(A, B, N, keep_stages=True, moduli_set=moduli_set)
    Ai = [[int(x) for x in row] for row in st["Aint"]]
    Bi = [[int(x) for x in row] for row in st["Bint"]]
    m, k, n = len(Ai), len(Bi), len(Bi[0])
    for i in range(m):
        for j in range(n):
            assert int(st["Cp"][i, j]) == sum(Ai[i][h] * Bi[h][j] for h in range(k))


def check_integer_inputs_exact(N=12, mode="accurate", moduli_set="hybrid"):
    """Integer inputs with small products: truncation is exact and C equals the
    exact product (a closed-form special case)."""
    A = integer_matrix(9, 33, 1000, 11)
    B = integer_matrix(33, 7, 1000, 12)
    C = ref.emulate(A, B, N, mode=mode, moduli_set=moduli_set)
    exact = np.array([[sum(int(A[i, h]) * int(B[h, j]) for h in range(33))
                       for j in range(7)] for i in range(9)], dtype=np.float64)
    assert np.array_equal(C, exact)


def check_error_bound(A, B, N, mode="accurate", moduli_set="hybrid"):
    """|C - AB| <= sum_h(|da||b| + |a||db| + |da||db|) + half an ulp of C, with
    |da_ih| < 2^-log2(mu_i) from truncation (exact rationals)."""
    C, st = ref.emulate(A, B, N, keep_stages=True, mode=mode, moduli_set=moduli_set)
    m, k = A.shape
    n = B.shape[1]
    for i in range(m):
        for j in range(n):
            exact = sum(Fraction(float(A[i, h])) * Fraction(float(B[h, j])) for h in range(k))
            da = Fraction(1, 2 ** int(st["sA"][i])) if st["sA"][i] >= 0 else Fraction(2 ** int(-st["sA"][i]))
            db = Fraction(1, 2 ** int(st["sB"][j])) if st["sB"][j] >= 0 else Fraction(2 ** int(-st["sB"][j]))
            bound = sum(da * abs(Fraction(float(B[h, j]))) + abs(Fraction(float(A[i, h]))) * db + da * db
                        for h in range(k))
            c = float(C[i, j])
            ulp = Fraction(math.ulp(c)) if c != 0 else Fraction(2) ** -1074
            assert abs(Fraction(c) - exact) <= bound + ulp / 2


def _e4m3_positive_values():
    """Every positive finite E4M3FN value, decoded from its bit fields: 1 sign,
    4 exponent (bias 7), 3 mantissa bits; exponent field 0 is subnormal and
    the all-ones pattern S.1111.111 is NaN."""
    vals = []
    for code in range(1, 0x7F):
        ex, man = code >> 3, code & 7
        vals.append(Fraction(man, 8) * Fraction(2) ** -6 if ex == 0
                    else (1 + Fraction(man, 8)) * Fraction(2) ** (ex - 7))
    return sorted(vals)


def check_fast_norms(A, B, N):
    """Fast mode (Section III-E, Cauchy-Schwarz): r_i is the squared norm of
    row i of the round-up bound operand, found here by brute force over the
    E4M3 value set with exact rationals; the Cauchy-Schwarz inequality then
    bounds every entry of the bound product, and the exponents follow the
    scale rule."""
    _, st = ref.emulate(A, B, N, keep_stages=True, mode="fast")
    grid = _e4m3_positive_values()

    def round_up(x):
        return Fraction(0) if x == 0 else next(v for v in grid if v >= x)

    def bars(X, E):
        mu = Fraction(2) ** (7 - int(E))
        return [round_up(mu * abs(Fraction(float(x)))) for x in X]

    m, k = A.shape
    n = B.shape[1]
    rows = [bars(A[i, :], st["EA"][i]) for i in range(m)]
    cols = [bars(B[:, j], st["EB"][j]) for j in range(n)]
    r = [sum(v * v for v in row) for row in rows]
    c = [sum(v * v for v in col) for col in cols]
    for i in range(m):
        assert Fraction(int(st["r18"][i]), 2 ** 18) == r[i]
    for j in range(n):
        assert Fraction(int(st["c18"][j]), 2 ** 18) == c[j]
    for i in range(m):
        for j in range(n):
            w = sum(a * b for a, b in zip(rows[i], cols[j]))
            assert w * w <= r[i] * c[j]
    P = st["P"]
    for x18, e in list(zip(st["r18"], st["e"])) + list(zip(st["c18"], st["f"])):
        check_scale_exponent_brute(P, [x18])
        assert ref.scale_exponent(x18, P) == e


def check_integer_conversion(A, B, N):
    """a'_ih = trunc(a_ih 2^log2(mu_i)) for every entry, with exact rationals
    (eq. def:A'), and b' likewise."""
    _, st = ref.emulate(A, B, N, keep_stages=True)
    for X, Xint, sh, rows in ((A, st["Aint"], st["sA"], True), (B, st["Bint"], st["sB"], False)):
        for i in range(X.shape[0]):
            for h in range(X.shape[1]):
                t = int(sh[i] if rows else sh[h])
                want = int(Fraction(float(X[i, h])) * Fraction(2) ** t)   # int() truncates
                assert int(Xint[i, h]) == want


def check_ufp(A):
    """ufp(max|a|) = 2^E means 2^E <= max|a| < 2^(E+1) (eq. def:mu'nu'), and
    the scaled maxima fall in [2^7, 2^8)."""
    EA = ref.ufp_exponents(A, axis=1)
    amax = np.max(np.abs(A), axis=1)
    for i in range(A.shape[0]):
        if amax[i] > 0:
            assert Fraction(2) ** int(EA[i]) <= Fraction(float(amax[i])) < Fraction(2) ** (int(EA[i]) + 1)
            assert 128 <= np.ldexp(amax[i], 7 - int(EA[i])) < 256


def check_smod():
    for p in (4, 5, 1024, 1089, 511):
        xs = np.arange(-3 * p, 3 * p, dtype=np.int64)
        v = ref.smod(xs, p)
        assert v.min() == -(p // 2) and v.max() == (p + 1) // 2 - 1
        assert np.all((xs - v) % p == 0)


def check_invariants(A, B, N, mode="accurate"):
    def em(X, Y):
        return ref.emulate(X, Y, N, mode=mode)

    C = em(A, B)
    assert np.array_equal(em(-A, B), -C)
    assert np.array_equal(em(A, -B), -C)
    assert np.array_equal(em(np.ldexp(A, 5), B), np.ldexp(C, 5))
    assert np.array_equal(em(A, np.ldexp(B, -3)), np.ldexp(C, -3))
    assert np.array_equal(em(B.T.copy(), A.T.copy()), C.T)
    perm = np.random.default_rng(5).permutation(A.shape[0])
    assert np.array_equal(em(A[perm], B), C[perm])


def check_fast_matches_accurate_when_tight(N):
    """Where every row of Abar and every column of Bbar is one constant vector,
    the Cauchy-Schwarz bound is attained (sum_h Abar Bbar = sqrt(r c)), so the
    two modes must pick the same exponents and give the same result.  Inputs:
    random signs times a power of two per row / column (Abar = Bbar = 128)."""
    rng = np.random.default_rng(31)
    m, k, n = 6, 40, 5
    A = rng.choice([-1.0, 1.0], (m, k)) * np.ldexp(1.0, rng.integers(-20, 20, (m, 1)))
    B = rng.choice([-1.0, 1.0], (k, n)) * np.ldexp(1.0, rng.integers(-20, 20, (1, n)))
    Cf, sf = ref.emulate(A, B, N, keep_stages=True, mode="fast")
    Ca, sa = ref.emulate(A, B, N, keep_stages=True)
    assert np.array_equal(sf["e"], sa["e"]) and np.array_equal(sf["f"], sa["f"])
    assert np.array_equal(sf["r18"], sa["r18"]) and np.array_equal(sf["c18"], sa["c18"])
    assert np.array_equal(Cf, Ca)


# ---- tests ----------------------------------------------------------------

def test_scale_exponent():
    rng = np.random.default_rng(3)
    for N in (1, 2, 3, 6, 12, 20, 33):
        P = math.prod(p for p, _, _ in ref.hybrid_moduli(N))
        vals = [0, 1, 2 ** 18, 2 ** 50, 3] + [int(v) for v in rng.integers(1, 2 ** 50, 200)]
        check_scale_exponent_brute(P, vals)


@pytest.mark.parametrize("N", [1, 2, 3, 6, 7, 12, 14])
def test_condition3(N):
    A, B = _small_problem(6, 5, 17, 2.0, 100 + N)
    check_condition3(A, B, N)


@pytest.mark.parametrize("N", [1, 2, 3, 6, 7, 12, 13])
def test_condition3_fast(N):
    A, B = _small_problem(6, 5, 17, 2.0, 150 + N)
    check_condition3(A, B, N, mode="fast")


@pytest.mark.parametrize("N,phi", [(13, 1.0), (6, 4.0)])
def test_fast_norms(N, phi):
    A, B = _small_problem(5, 4, 14, phi, 160 + N)
    A[1, :] = 0.0
    A[2, 3] = 5e-324
    check_fast_norms(A, B, N)


@pytest.mark.parametrize("N", [1, 7, 12, 13])
def test_fast_matches_accurate_when_tight(N):
    check_fast_matches_accurate_when_tight(N)


# Karatsuba-only moduli (Section III-B list, R14): 513 = 3^3 19, 512 = 2^9 and
# 505 = 5 101 are among the first five, so N = 5 covers the moduli whose
# digits reach 16 and the ones sharing factors with 15 and 16
@pytest.mark.parametrize("N", [1, 2, 5, 12, 13])
def test_karatsuba_only_pins(N):
    A, B = _small_problem(5, 6, 19, 1.5, 170 + N)
    check_condition3(A, B, N, moduli_set="karatsuba")
    check_residue_products(A, B, N, moduli_set="karatsuba")
    check_crt_is_exact_product(A, B, N, moduli_set="karatsuba")
    check_error_bound(A[:3, :], B[:, :3], N, moduli_set="karatsuba")
    check_condition3(A, B, N, mode="fast", moduli_set="karatsuba")


def test_karatsuba_only_integer_inputs_and_accuracy():
    # P/2 > 2^115 from N = 13 on (Section III-B), so 13 Karatsuba-only moduli
    # reach the accuracy that 12 hybrid moduli reach (P/2 > 2^110)
    check_integer_inputs_exact(13, moduli_set="karatsuba")
    A, B = _small_problem(24, 20, 1500, 0.5, 510)
    hi, lo = dd_dot_rows(A, B)
    err13 = normalised_error(ref.emulate(A, B, 13, moduli_set="karatsuba"), hi, lo,
                             np.abs(A), np.abs(B))
    err_h12 = normalised_error(ref.emulate(A, B, 12), hi, lo, np.abs(A), np.abs(B))
    assert err13 <= 1e-15 and err_h12 <= 1e-15, (err13, err_h12)
    for moduli_set in ("hybrid", "karatsuba"):
        with pytest.raises(ValueError):
            ref.moduli_table(10 ** 4, moduli_set)
    with pytest.raises(ValueError):
        ref.moduli_table(3, "binary")


# INT8 arm (Section II list, R15): 256 = 2^8 and 255 = 3 5 17 come first; the
# residues are the INT8 operands themselves
@pytest.mark.parametrize("N", [1, 2, 5, 14, 16])
def test_int8_arm_pins(N):
    A, B = _small_problem(5, 6, 19, 1.5, 180 + N)
    check_condition3(A, B, N, moduli_set="int8")
    check_residue_products(A, B, N, moduli_set="int8")
    check_crt_is_exact_product(A, B, N, moduli_set="int8")
    check_error_bound(A[:3, :], B[:, :3], N, moduli_set="int8")
    check_condition3(A, B, N, mode="fast", moduli_set="int8")
    _, st = ref.emulate(A, B, N, keep_stages=True, moduli_set="int8")
    for pm in st["per_modulus"]:
        assert len(pm["dA"]) == 1 and np.array_equal(pm["dA"][0], pm["uA"])
        assert pm["uA"].min() >= -128 and pm["uA"].max() <= 127


def test_int8_arm_accuracy_and_int32_limit():
    # P/2 > 2^109 from N = 14 on (Section II): 14 INT8 moduli reach FP64-level
    # accuracy on narrow-range inputs, 13 do not
    check_integer_inputs_exact(14, moduli_set="int8")
    A, B = _small_problem(24, 20, 1500, 0.5, 520)
    hi, lo = dd_dot_rows(A, B)
    e14 = normalised_error(ref.emulate(A, B, 14, moduli_set="int8"), hi, lo, np.abs(A), np.abs(B))
    e13 = normalised_error(ref.emulate(A, B, 13, moduli_set="int8"), hi, lo, np.abs(A), np.abs(B))
    assert e14 <= 1e-15 < e13, (e13, e14)
    # all residues -128 over a chunk of 2^16: 2^30, inside INT32; the check
    # refuses a chunk whose sum would not be
    k = 2 ** 16
    u = np.full((1, k), -128, dtype=np.int64)
    got = ref.residue_product_fp8([u], [u.T.copy()], 251, "int8", 0)
    assert int(got[0, 0]) == ref.smod(2 ** 30, 251)
    with pytest.raises(ArithmeticError):
        ref.residue_product_fp8([np.full((1, 2 ** 17), -128)], [np.full((2 ** 17, 1), -128)],
                                251, "int8", 0, chunk=2 ** 17)


def test_bound_dominates():
    A, B = _small_problem(5, 4, 13, 3.0, 7)
    A[2, :] = 0.0
    check_bound_dominates(A, B, 12)


@pytest.mark.parametrize("N", [1, 3, 6, 7, 12, 16])
def test_residue_products(N):
    A, B = _small_problem(5, 6, 19, 1.0, 200 + N)
    check_residue_products(A, B, N)


@pytest.mark.parametrize("N", [1, 2, 6, 12, 20])
def test_crt_exact_product(N):
    A, B = _small_problem(4, 5, 23, 1.0, 300 + N)
    check_crt_is_exact_product(A, B, N)


def test_integer_inputs_exact():
    check_integer_inputs_exact(12)
    check_integer_inputs_exact(12, mode="fast")


@pytest.mark.parametrize("N,phi", [(12, 0.5), (6, 1.0), (3, 4.0), (12, 4.0)])
def test_error_bound(N, phi):
    A, B = _small_problem(4, 4, 21, phi, 400 + N)
    check_error_bound(A, B, N)


@pytest.mark.parametrize("N,phi", [(13, 0.5), (6, 1.0), (13, 4.0)])
def test_error_bound_fast(N, phi):
    A, B = _small_problem(4, 4, 21, phi, 450 + N)
    check_error_bound(A, B, N, mode="fast")


@pytest.mark.parametrize("phi", [0.5, 4.0])
def test_integer_conversion(phi):
    A, B = _small_problem(5, 4, 12, phi, 700)
    A[0, 0] = 5e-324
    check_integer_conversion(A, B, 12)
    check_integer_conversion(A, B, 20)


def test_smod():
    check_smod()


def test_ufp():
    A, _ = _small_problem(7, 1, 30, 4.0, 800)
    A[2, 3] = 5e-324
    A[2, :3] = 0.0
    A[2, 4:] = 0.0
    check_ufp(A)


def test_invariants():
    A, B = _small_problem(11, 9, 37, 1.0, 17)
    check_invariants(A, B, 12)
    check_invariants(A, B, 13, mode="fast")


def test_residue_product_chunked_k():
    # k > 2^16 in the digit route is summed in exact chunks (reading R12):
    # all-16 digits at k = 2^16 + 5 make every chunk product reach 2^24
    k = 2 ** 16 + 5
    d = [np.full((1, k), 16, dtype=np.int64), np.full((1, k), 16, dtype=np.int64)]
    dB = [x.T.copy() for x in d]
    got = ref.residue_product_fp8(d, dB, 1089, "square", 33)
    exact = (33 * 256 * k + 33 * 256 * k + 256 * k)
    assert int(got[0, 0]) == ref.smod(exact, 1089)


def test_zero_and_nonfinite_lines():
    A, B = _small_problem(5, 4, 8, 1.0, 21)
    A[1, :] = 0.0
    A[3, 2] = np.inf
    B[4, 0] = np.nan
    C, st = ref.emulate(A, B, 12, keep_stages=True)
    assert np.all(C[1, 1:] == 0.0) and not np.any(np.signbit(C[1, 1:]))
    assert np.all(np.isnan(C[3, :])) and np.all(np.isnan(C[:, 0]))
    assert st["e"][1] == 0 and st["EA"][1] == 0
    good = C[[0, 2, 4]][:, 1:]
    A2 = A.copy(); A2[3, 2] = 0.0
    B2 = B.copy(); B2[4, 0] = 0.0
    assert np.array_equal(ref.emulate(A2, B2, 12)[[0, 2, 4]][:, 1:], good)


def test_accuracy_full_moduli():
    # N = 12 gives about 55 effective bits relative to the row and column
    # maxima (Table 2).  For narrow-range inputs (phi = 0.5) that is FP64-level
    # normalised error; a wider spread of magnitudes needs more moduli
    # (measured: phi = 2 -> 13, phi = 4 -> 14).
    for phi, N in ((0.5, 12), (2.0, 13), (4.0, 14)):
        A, B = _small_problem(24, 20, 1500, phi, 500)
        hi, lo = dd_dot_rows(A, B)
        err = normalised_error(ref.emulate(A, B, N), hi, lo, np.abs(A), np.abs(B))
        assert err <= 1e-15, (phi, N, err)
        err_less = normalised_error(ref.emulate(A, B, N - 1), hi, lo, np.abs(A), np.abs(B))
        assert err_less > 1e-15, (phi, N - 1, err_less)
    # and the error falls as moduli are added
    errs = []
    A, B = _small_problem(16, 16, 600, 1.0, 501)
    hi, lo = dd_dot_rows(A, B)
    for N in (6, 8, 10, 12):
        errs.append(normalised_error(ref.emulate(A, B, N), hi, lo, np.abs(A), np.abs(B)))
    assert errs[0] > errs[1] > errs[2] > errs[3]


def test_accuracy_fast_mode():
    # Fast mode's Cauchy-Schwarz bound is looser than the bound product, so it
    # may need one more modulus for the same accuracy (Section V-A uses 13 for
    # fast mode against 12 for accurate mode).  Measured on these inputs:
    # phi = 0.5 -> equal errors at N = 12, phi = 2 -> fast needs N = 13.
    A, B = _small_problem(24, 20, 1500, 0.5, 500)
    hi, lo = dd_dot_rows(A, B)
    err = normalised_error(ref.emulate(A, B, 12, mode="fast"), hi, lo, np.abs(A), np.abs(B))
    assert err <= 1e-15, err
    A, B = _small_problem(24, 20, 1500, 2.0, 500)
    hi, lo = dd_dot_rows(A, B)
    acc12 = normalised_error(ref.emulate(A, B, 12), hi, lo, np.abs(A), np.abs(B))
    fast12 = normalised_error(ref.emulate(A, B, 12, mode="fast"), hi, lo, np.abs(A), np.abs(B))
    fast13 = normalised_error(ref.emulate(A, B, 13, mode="fast"), hi, lo, np.abs(A), np.abs(B))
    assert fast12 > 1e-15 >= fast13 and fast12 >= acc12, (acc12, fast12, fast13)


def test_dd_reference_against_rationals():
    A, B = _small_problem(3, 4, 50, 3.0, 600)
    hi, lo = dd_dot_rows(A, B)
    for i in range(3):
        for j in range(4):
            exact = sum(Fraction(float(A[i, h])) * Fraction(float(B[h, j])) for h in range(50))
            err = abs(Fraction(float(hi[i, j])) + Fraction(float(lo[i, j])) - exact)
            scale = sum(abs(Fraction(float(A[i, h])) * Fraction(float(B[h, j]))) for h in range(50))
            assert err <= scale * Fraction(1, 2 ** 100)


def test_rounding_helper_subnormal():
    # one correctly rounded step: 3 * 2^-1076 = 0.75 * 2^-1074 -> 2^-1074;
    # 2^53 + 1 scaled into the subnormal range rounds to even
    assert ref._rn_scaled(3, 1076) == 5e-324
    assert ref._rn_scaled(1, 1075) == 0.0                   # tie -> even (0)
    assert ref._rn_scaled(3, 1075) == 2 * 5e-324            # tie 1.5 -> 2
    assert ref._rn_scaled(-1, 2000) == 0.0 and math.copysign(1, ref._rn_scaled(-1, 2000)) < 0
    assert ref._rn_scaled(2 ** 53 + 1, 0) == 2.0 ** 53
    assert ref._rn_scaled(2 ** 53 + 3, 0) == 2.0 ** 53 + 4
    assert ref._rn_scaled(1, -1024) == math.inf


@pytest.mark.parametrize("mode,moduli_set,N", [("accurate", "hybrid", 12), ("fast", "hybrid", 13),
                                               ("accurate", "int8", 15),
                                               ("accurate", "karatsuba", 5)])
def test_scaling_lines_equals_full_scaling(mode, moduli_set, N):
    # the line-restricted scaling (used where the whole bound product is too
    # large to form on the CPU) gives every sampled line the exponents of the
    # full oracle, and the sampled outputs equal the full emulation's
    A, B = _small_problem(37, 29, 70, 2.0, 31)
    A[4, :] = 0.0
    A[6, 3] = np.inf
    B[:, 7] = 0.0
    B[11, 9] = np.nan
    A[9] *= 2.0 ** 40
    B[:, 2] *= 2.0 ** -30
    rows = np.array([0, 4, 6, 9, 36, 9])
    cols = np.array([28, 2, 7, 9, 0])
    full = ref.scaling(A, B, N, mode=mode, moduli_set=moduli_set)
    part = ref.scaling_lines(A, B, N, rows, cols, mode=mode, moduli_set=moduli_set)
    for key, sel in (("EA", rows), ("e", rows), ("sA", rows), ("r18", rows), ("badA", rows),
                     ("EB", cols), ("f", cols), ("sB", cols), ("c18", cols), ("badB", cols)):
        assert np.array_equal(part[key], full[key][sel]), key
    want, _ = ref.products(full, rows, cols)
    got, _ = ref.products(part, slice(None), slice(None))
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.array_equal(np.nan_to_num(got).view(np.int64), np.nan_to_num(want).view(np.int64))
    # one bound serves every number of moduli
    b = ref.line_bounds(A, B, rows, cols, mode)
    for N2 in (N - 1, N + 1):
        f2 = ref.scaling(A, B, N2, mode=mode, moduli_set=moduli_set)
        p2 = ref.scaling_from_bounds(b, N2, moduli_set)
        assert np.array_equal(p2["sA"], f2["sA"][rows]) and np.array_equal(p2["sB"], f2["sB"][cols])
