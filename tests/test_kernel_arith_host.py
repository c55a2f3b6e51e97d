"""The FP32 steps of the residue-product kernels, modelled in numpy float32 on
the host (float32 products and rint round to nearest-even as the GPU's do;
the fused multiply-adds there are exact, so they are modelled in integers):

* the Karatsuba fold: y = (x - rint(x / p) p) mul, then y - rint(y / p) p,
  for exact integer accumulators |x| <= 2^23 + 259 (a pass of k = 2^15
  products of digits |d| <= 16 on top of a folded value), with the two
  multipliers of every modulus: the result is congruent to mul x and at most
  p/2 + 2 in magnitude, so the next pass stays exact below 2^24;
* the square fold: x - rint(x / s) s for |x| <= 2^24 (two passes of cross
  products), congruent to x modulo s and at most s/2 + 2;
* the epilogue remainder (float quotient estimate, two corrections) for the
  largest values each kind produces: |v| <= 16 (2^23 + 259) (Karatsuba,
  final multiplier), 2^24 + s (s/2 + 2) (squares), 2^29 (INT8 sums of 2^15
  products of residues in [-128, 127]) -- equal to the exact symmetric
  remainder.

The largest magnitudes are covered exhaustively near the top of each range
(where the estimate errors are largest) and by random samples elsewhere, for
every modulus of all three lists up to N = 33."""
import numpy as np
import pytest

from oracle import ozaki2_ref as ref

RNG = np.random.default_rng(9100)


def _inv(p):
    return np.float32(1.0) / np.float32(p)


def _est(x, p):
    """rint(x * fl(1/p)) with x already an exact float32 integer."""
    return np.rint(x.astype(np.float32) * _inv(p)).astype(np.int64)


def _sym(v, p):
    r = np.mod(v, p)
    return np.where(r > p - 1 - p // 2, r - p, r)


def _values(top, n_top, n_rand):
    hi = np.arange(top - n_top, top + 1, dtype=np.int64)
    rnd = RNG.integers(-top, top + 1, n_rand, dtype=np.int64)
    return np.concatenate([hi, -hi, rnd, np.arange(-4096, 4097, dtype=np.int64)])


def _inv_mod(a, p):
    return pow(int(a) % p, -1, p)


def _karatsuba_multipliers(p):
    s = lambda v: int(_sym(np.int64(v), p))
    if np.gcd(p, 15) == 1:
        return s(15), s(-16 * _inv_mod(15, p)), s(-15)
    assert p % 2 == 1
    return s(-16), s(-15 * _inv_mod(16, p)), s(16)


def _smod_i32(v, p):
    # the epilogue's remainder: float estimate, then one correction each way
    assert np.all(np.abs(v) < 2 ** 31)
    r = v - _est(v, p) * p
    lo, hi = -(p >> 1), p - 1 - (p >> 1)
    r = np.where(r > hi, r - p, r)
    return np.where(r < lo, r + p, r)


def _moduli(kind):
    out = set()
    for name in ("hybrid", "karatsuba", "int8"):
        for p, k, s in ref.moduli_table(33, name):
            if k == kind:
                out.add((p, s))
    return sorted(out)


@pytest.mark.parametrize("p", [p for p, _ in _moduli("karatsuba")])
def test_karatsuba_fold_exact_and_bounded(p):
    x = _values(2 ** 23 + 259, 1 << 16, 1 << 16)
    assert np.all(x.astype(np.float32).astype(np.int64) == x)
    a, b, c = _karatsuba_multipliers(p)
    for mul in (a, b):
        y = (x - _est(x, p) * p) * mul
        assert np.all(np.abs(y) < 2 ** 24)
        t = y - _est(y, p) * p
        assert np.all(np.abs(t) <= p // 2 + 2)
        assert np.all(np.mod(t - mul * x, p) == 0)
    v = c * x
    assert np.array_equal(_smod_i32(v, p), _sym(v, p))


@pytest.mark.parametrize("p,s", _moduli("square"))
def test_square_fold_exact_and_bounded(p, s):
    x = _values(2 ** 24, 1 << 17, 1 << 16)
    t = x - _est(x, s) * s
    assert np.all(np.abs(t) <= s // 2 + 2)
    assert np.all(np.mod(t - x, s) == 0)
    acc = t * s
    assert np.all(np.abs(acc) <= s * (s // 2 + 2))
    # the third pass adds at most 2^23; the epilogue reduces modulo s^2
    v = _values(2 ** 24 + s * (s // 2 + 2), 1 << 16, 1 << 16)
    assert np.array_equal(_smod_i32(v, p), _sym(v, p))


@pytest.mark.parametrize("p", [p for p, _ in _moduli("int8")])
def test_int8_epilogue_remainder(p):
    v = _values(2 ** 29, 1 << 18, 1 << 17)
    assert np.array_equal(_smod_i32(v, p), _sym(v, p))
    # a later k chunk adds the stored plane value (|r| <= p/2) to a new one
    w = np.arange(-p, p + 1, dtype=np.int64)
    assert np.array_equal(_smod_i32(w, p), _sym(w, p))
