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
every modulus of all three lists up to N = 33.

And the residue pass of the quantization kernel (x mod p for the scaled
integers): the FP64 step x - rint(x fl(1/R)) R, for R = p alone or for
R = p p' (two consecutive moduli of one kind), for integers |x| < 2^53 and
|x| = mant 2^10 < 2^63 near ties, then one FP32 step per modulus with no
further correction for odd p (one for even p) must give the symmetric residue;
likewise for the later multiplication by 2^t mod p; and the square digit
rint(u fl(1/s)) must equal round(u / s) with ties away from zero for odd s.
The bound operands' E4M3 round-up code 8 e + 48 + Q is checked against the
oracle's round-up over all E4M3 values of rows from subnormal to huge, and
the residue pass's integer x 2^tt (x = trunc(a 2^(s - tt))) against the
oracle's a' = trunc(a 2^s)."""
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


def _all_moduli():
    out = set()
    for name in ("hybrid", "karatsuba", "int8"):
        for p, _, _ in ref.moduli_table(33, name):
            out.add(p)
    return sorted(out)


def _fp32_step(f, p):
    """f - rint(f fl(1/p)) p, then for even p +p/2 moved to -p/2."""
    r = f - _est(f, p) * p
    if p % 2 == 0:
        r = np.where(r > p - 1 - p // 2, r - p, r)
    return r


def _near_ties(p, top, count):
    """Integers below `top` in magnitude whose residue sits at or next to
    +-p/2, the wrap point, or 0."""
    q = RNG.integers(0, top // p - 1, count, dtype=np.int64)
    off = np.array([-(p // 2) - 1, -(p // 2), -(p // 2) + 1, -1, 0, 1, p // 2 - 1, p // 2,
                    p // 2 + 1, (p + 1) // 2], dtype=np.int64)
    x = (q[:, None] * p + off[None, :]).ravel()
    x = x[np.abs(x) < top]
    return np.concatenate([x, -x])


@pytest.mark.parametrize("p", _all_moduli())
def test_residue_pass_reduction(p):
    inv = np.float64(1.0) / np.float64(p)
    # |x| < 2^53: any integer
    small = np.concatenate([_near_ties(p, 2 ** 53, 1 << 14),
                            RNG.integers(-2 ** 53 + 1, 2 ** 53, 1 << 15, dtype=np.int64),
                            np.arange(-4 * p, 4 * p + 1, dtype=np.int64)])
    # mant 2^10 with mant < 2^53: chosen near ties through mant = x / 2^10
    mant = _near_ties(p, 2 ** 53, 1 << 14) // p * p
    big = np.concatenate([mant * 1024, (mant + RNG.integers(0, p, mant.size)) * 1024,
                          np.array([(2 ** 53 - 1) * 1024, -(2 ** 53 - 1) * 1024])])
    for x in (small, big):
        xf = x.astype(np.float64)
        assert np.all(xf.astype(np.int64) == x)            # exact doubles
        q = np.rint(xf * inv).astype(np.int64)
        f = x - q * p                                       # the exact fma
        assert np.all(np.abs(f) < 2 ** 15)
        assert np.array_equal(_fp32_step(f, p), _sym(x, p))


def _pairs():
    """The moduli the residue pass reduces two at a time: consecutive moduli of
    one kind, paired from the kind's first (a run of odd length leaves its
    last modulus alone).  The pairs of N = 33 contain those of every N."""
    out = set()
    for name in ("hybrid", "karatsuba", "int8"):
        table = ref.moduli_table(33, name)
        l = 0
        while l < len(table):
            end = l
            while end < len(table) and table[end][1] == table[l][1]:
                end += 1
            for a in range(l, end - 1, 2):
                out.add((table[a][0], table[a + 1][0]))
            l = end
    return sorted(out)


@pytest.mark.parametrize("p,p2", _pairs())
def test_residue_pass_paired_reduction(p, p2):
    # one FP64 step modulo R = p p2 (< 2^21), then the FP32 step of each modulus
    R = p * p2
    assert R < 2 ** 21
    inv = np.float64(1.0) / np.float64(R)
    small = np.concatenate([_near_ties(p, 2 ** 53, 1 << 13), _near_ties(p2, 2 ** 53, 1 << 13),
                            _near_ties(R, 2 ** 53, 1 << 13),
                            RNG.integers(-2 ** 53 + 1, 2 ** 53, 1 << 14, dtype=np.int64),
                            np.arange(-3 * R, 3 * R + 1, 97, dtype=np.int64)])
    mant = np.concatenate([_near_ties(q, 2 ** 53, 1 << 12) // q * q for q in (p, p2, R)])
    big = np.concatenate([mant * 1024, (mant + RNG.integers(0, R, mant.size)) * 1024,
                          np.array([(2 ** 53 - 1) * 1024, -(2 ** 53 - 1) * 1024])])
    for x in (small, big):
        xf = x.astype(np.float64)
        assert np.all(xf.astype(np.int64) == x)            # exact doubles
        q = np.rint(xf * inv).astype(np.int64)
        f = x - q * R                                       # the exact fma
        assert np.all(np.abs(f) < 2 ** 20 + 2 ** 11)
        assert np.array_equal(_fp32_step(f, p), _sym(x, p))
        assert np.array_equal(_fp32_step(f, p2), _sym(x, p2))


@pytest.mark.parametrize("p", _all_moduli())
def test_residue_pass_power_step(p):
    # u in the symmetric range times every tabulated 2^t mod p
    u = np.arange(-(p // 2), p - p // 2, dtype=np.int64)
    pw = np.unique([pow(2, t, p) for t in range(1, 192)]).astype(np.int64)
    prod = (u[:, None] * pw[None, :]).ravel()
    assert np.all(np.abs(prod) < 2 ** 20)
    assert np.array_equal(_fp32_step(prod, p), _sym(prod, p))


def _residue_integer(a, s):
    """The residue pass's integer as the kernel forms it: t = frexp exponent
    - 53 + s (clamped below 192), tt = max(t - 10, 0), x = trunc(a 2^(s - tt))
    + 0 for finite nonzero a, else +0; a' = x 2^tt."""
    _, E = np.frexp(a)
    nz = np.isfinite(a) & (a != 0)
    t = np.where(nz, np.minimum(E - 53 + s, 191), 0)
    tt = np.where(t > 10, t - 10, 0)
    with np.errstate(over="ignore", invalid="ignore"):
        x = np.trunc(np.ldexp(a, s - tt)) + 0.0
    return np.where(nz, x, 0.0), tt


def test_residue_integer_formation():
    # a' = trunc(a 2^s) (eq. def:A') from x 2^tt, over doubles from subnormal
    # to huge and shifts giving t from -120 (a' = 0) to 181
    for _ in range(40):
        E = int(RNG.integers(-1074, 1024))
        a = np.ldexp(RNG.random(2048) + 0.5, E - RNG.integers(0, 60, 2048))
        a = np.concatenate([a, np.ldexp(RNG.integers(1, 1 << 52, 64).astype(np.float64), -1074)])
        a = a[np.isfinite(a) & (a > 0)]
        a = np.concatenate([a, -a, [0.0, -0.0]])
        _, Ea = np.frexp(np.max(np.abs(a)))
        for t_top in (-120, -1, 0, 1, 10, 11, 53, 120, 181):
            s = t_top - (int(Ea) - 53)                  # the largest input gets t = t_top
            x, tt = _residue_integer(a, s)
            assert np.all(np.abs(x) < 2.0 ** 63) and np.all(np.trunc(x) == x)
            assert not np.any(np.signbit(x) & (x == 0))  # never -0
            want = ref.to_integers(a[None, :], np.array([s]), axis=0)[0]
            with np.errstate(over="ignore"):
                got = np.ldexp(x, tt)
            ok = np.isfinite(want)
            assert np.array_equal(got[ok], want[ok]), (E, t_top)


def _round_up_code(a, sh):
    """The bound operands' E4M3 round-up as the kernel computes it: with
    fl = frexp exponent - 1 + sh = floor(log2 |a| 2^sh) and e = max(fl, -6),
    Q = max(ceil(|a| 2^(sh + 3 - e)), 1) and the code is 8 e + 48 + Q."""
    _, E = np.frexp(a)
    e = np.maximum(E - 1 + sh, -6)
    Q = np.maximum(np.ceil(np.ldexp(np.abs(a), sh + 3 - e)), 1.0)
    return 8 * e + 48 + Q.astype(np.int64)


def test_bound_round_up_code_formula():
    # rows with ufp exponent E (sh = 7 - E), from subnormal to huge doubles:
    # every E4M3 value of the row's range, its neighbours one double ulp
    # away, random magnitudes over 80 binades, and subnormal doubles
    grid = ref.E4M3_NONNEG[1:]
    for E in list(range(-1074, -1000, 3)) + list(range(-1000, 1024, 37)) + [1023]:
        sh = 7 - E
        with np.errstate(over="ignore"):    # grid values past the largest double
            top = np.ldexp(1.0, E) * (1.0 + RNG.random(64))        # the row maxima
            on = np.ldexp(grid, -sh)                                 # E4M3 values of the row
            near = np.concatenate([on, np.nextafter(on, 0.0), np.nextafter(on, np.inf)])
            end = np.ldexp(2.0, E)                                   # the row's binade end
        rnd = np.ldexp(RNG.random(4096) + 0.5, E - RNG.integers(0, 80, 4096))
        sub = np.ldexp(RNG.integers(1, 1 << 20, 256).astype(np.float64), -1074)
        a = np.concatenate([top, near, rnd, sub])
        a = a[(a > 0) & (a < end) & np.isfinite(a)]
        a = np.concatenate([a, -a])
        want = ref.e4m3_encode_exact(ref.round_up_e4m3(np.ldexp(np.abs(a), sh), a != 0))
        got = _round_up_code(a, sh)
        assert np.array_equal(got, want.astype(np.int64)), E


@pytest.mark.parametrize("p,s", [(p, s) for p, s in _moduli("square") if s % 2 == 1])
def test_square_digit_odd_radix(p, s):
    u = np.arange(-(p // 2), p - p // 2, dtype=np.int64)
    got = np.rint(u.astype(np.float32) * _inv(s)).astype(np.int64)
    want = np.sign(u) * ((2 * np.abs(u) + s) // (2 * s))    # ties away from zero
    assert np.array_equal(got, want)
    assert np.all(np.abs(got) <= 16) and np.all(np.abs(u - s * got) <= 16)

