"""Pins for the oracle's FP8 E4M3 handling and the digit splits.

The E4M3 decode table is checked against torch's float8_e4m3fn conversion (a
library routine); the round-up cast against brute force with exact rationals;
the digit splits exhaustively over every residue of every modulus."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import ozaki2_ref as ref


def test_decode_matches_torch():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    tv = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([ref.e4m3_decode(c) for c in range(256)])
    both_nan = np.isnan(tv) & np.isnan(mine)
    assert np.all(both_nan | (tv == mine))
    assert np.sum(np.isnan(mine)) == 2          # S.1111.111 only


def test_format_facts():
    # Section III-A: consecutive integers -16..16 are exact; 17 is not
    vals = set(ref.E4M3_NONNEG.tolist())
    assert all(float(i) in vals for i in range(0, 17))
    assert 17.0 not in vals
    assert ref.E4M3_MAX == 448.0 and ref.E4M3_MIN_POS == 2.0 ** -9
    assert np.all(np.diff(ref.E4M3_NONNEG) > 0)


def _ru_brute(x: Fraction) -> float:
    for v in ref.E4M3_NONNEG:
        if Fraction(v) >= x:
            return float(v)
    raise AssertionError


def test_round_up_brute_force():
    rng = np.random.default_rng(1)
    e = rng.uniform(-14, 8, 4000)
    x = np.ldexp(rng.uniform(1, 2, 4000), np.floor(e).astype(int))
    x = np.concatenate([x, ref.E4M3_NONNEG[1:], ref.E4M3_NONNEG[1:] * (1 + 2 ** -40),
                        [2.0 ** -9, 2.0 ** -10, 255.9, 256.0]])
    x = x[x <= 256]
    got = ref.round_up_e4m3(x, x != 0)
    for xi, gi in zip(x, got):
        assert gi == _ru_brute(Fraction(float(xi)))


def test_round_up_underflowed_inputs():
    # an exact value below 2^-1022 may reach the cast as 0 or a rounded
    # subnormal; its round-up is still 2^-9 because the input was nonzero
    x = np.array([0.0, 5e-324, 0.0])
    nz = np.array([True, True, False])
    assert list(ref.round_up_e4m3(x, nz)) == [2.0 ** -9, 2.0 ** -9, 0.0]


def test_bound_operand_dominates_and_fits():
    rng = np.random.default_rng(2)
    A = (rng.random((16, 40)) - 0.5) * np.exp(4 * rng.standard_normal((16, 40)))
    A[3, :] = 0.0
    A[5, 7] = 5e-324
    EA = ref.ufp_exponents(A, axis=1)
    B = np.ones((40, 1))
    Abar, _ = ref.bound_operands(A, B, EA, np.zeros(1, dtype=np.int64))
    for i in range(16):
        for h in range(40):
            exact = Fraction(abs(float(A[i, h]))) * Fraction(2) ** (7 - int(EA[i]))
            assert Fraction(float(Abar[i, h])) >= exact     # round-up
            assert float(Abar[i, h]) <= 256.0               # mu'|a| < 2^8
            assert float(Abar[i, h]) == _ru_brute(exact)
    # ufp: 2^E <= max|a| < 2^(E+1)
    amax = np.max(np.abs(A), axis=1)
    for i in range(16):
        if amax[i] > 0:
            assert 2.0 ** EA[i] <= amax[i] < 2.0 ** (EA[i] + 1)
        else:
            assert EA[i] == 0


@pytest.mark.parametrize("p,kind,s", ref.hybrid_moduli(34) + ref.moduli_table(33, "karatsuba"))
def test_digits_exhaustive(p, kind, s):
    u = np.arange(-(p // 2), (p + 1) // 2, dtype=np.int64)
    d = ref.digit_slices(u, kind, s)
    for x in d:
        assert np.max(np.abs(x)) <= 16          # exact in E4M3, and k*16*16 <= 2^24
        ref.e4m3_encode_exact(x.astype(np.float64))
    if kind == "square":
        x1, x2 = d
        assert np.all(s * x1 + x2 == u)
        # round-to-nearest split: |x2| <= s/2
        assert np.all(2 * np.abs(x2) <= s)
    else:
        x1, x2, x3 = d
        assert np.all(16 * x1 + x2 == u)
        assert np.all(x3 == x1 + x2)
        assert np.all(x1 == np.sign(u) * np.ceil(np.abs(u) / 16))


@pytest.mark.parametrize("p,kind,s", ref.moduli_table(33, "int8"))
def test_int8_operands_exhaustive(p, kind, s):
    # INT8 arm: the operand is the residue, in [-128, 127] for every p <= 256
    u = np.arange(-(p // 2), (p + 1) // 2, dtype=np.int64)
    (x,) = ref.digit_slices(u, kind, s)
    assert np.array_equal(x, u) and x.min() >= -128 and x.max() <= 127
    assert np.array_equal(ref.smod(u, p), u)


def test_max_digit_is_16():
    # the bound 16 is reached (so it is tight) for 1089, 1024 and 511..487;
    # the smaller moduli stay at 15 or below
    tops = {}
    for p, kind, s in ref.hybrid_moduli(33):
        u = np.arange(-(p // 2), (p + 1) // 2, dtype=np.int64)
        tops[p] = max(int(np.max(np.abs(x))) for x in ref.digit_slices(u, kind, s))
    big = {1089, 1024, 511, 509, 503, 499, 491, 487}
    assert all(tops[p] == 16 for p in big)
    assert all(v <= 15 for p, v in tops.items() if p not in big)


def test_encode_exact_rejects_and_signs():
    codes = ref.e4m3_encode_exact(np.array([0.0, -1.0, 16.0, -16.0, 1.5]))
    assert [ref.e4m3_decode(int(c)) for c in codes] == [0.0, -1.0, 16.0, -16.0, 1.5]
    assert codes[0] == 0x00
    with pytest.raises(ValueError):
        ref.e4m3_encode_exact(np.array([17.0]))
