"""CPU oracle for DGEMM emulation by the Ozaki-II scheme with FP8 quantization
(Uchino, Ozaki, Imamura, arXiv 2603.10634).

TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct reference
that the HIP library is checked against.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code, table or constant generator with the HIP library.

Every step follows the paper in its order and notation (sections cited per
function).  Arithmetic is exact throughout:

* integer-valued matrices are held in float64 and multiplied with numpy's
  float64 matmul only where every partial sum is an integer of magnitude
  below 2^53, so the library product is exact whatever order it sums in;
* remainders of float64 integers use C fmod, which is exact for all inputs;
* the Chinese-remainder sum and the final rounding use Python integers and
  CPython's correctly rounded int/int true division.

Readings of the paper taken here (where it is silent, ambiguous or garbled):

R1  bound operands use |A| and |B|: the bound chain needs absolute values.
R2  "max_h cbar_ih" is the maximum over the row i of the bound product
    (column maximum for nu).
R3  scale rule: e_i is the largest integer e with 2^(2e+1) * r_i <= P - 1,
    where r_i is the row maximum of the bound product.  This is what the
    implementation formula for log2(mu) (Section III-E) computes in exact
    arithmetic; it guarantees condition (3) because cbar_ij <= sqrt(r_i c_j).
R4  the bound product is taken exactly (Abar*Bbar has no rounding here).  The
    paper computes it in FP32 on FP8 matrix units and inflates it by
    (1 + k 2^-24); that value depends on the hardware's summation order, and
    on gfx950 the inflation is not even an upper bound (the FP8 MFMA truncates
    products inside groups of 8 terms).  Taking the exact product makes the
    scale exponents a function of the inputs alone.  Any implementation that
    settles a line from an inexact bound must therefore prove that the exact
    value gives the same exponent (else recompute it exactly) to agree here.
R5  int(.) in the scale formula is floor (its argument may be negative).
R6  zero rows/columns: exponent 0, scale exponent 0; their outputs are +0.
R7  symmetric modulo: smod(x, p) lies in [-floor(p/2), ceil(p/2) - 1].
R8  round() in the square-modulus digit split rounds half away from zero.
R9  rows of op(A) / columns of op(B) holding a non-finite value are treated as
    zero during quantization and give NaN in every output they touch.
R10 final rounding: one round-to-nearest-even of the exact rational C' 2^-t
    (subnormals included), then C = alpha*Chat (+ beta*C_in), each operation
    rounded to nearest; C_in is not read when beta == 0.
R11 FP8 is OCP E4M3FN (max 448): the bound operands reach 256.
R12 k > 2^16: the residue products are summed in chunks of 2^16 and reduced
    modulo p (the modulo is linear), which is exact.
R13 fast mode (Section III-E names it and says only that it bounds the sum of
    |a'||b'| by the Cauchy-Schwarz inequality): r_i is the squared Euclidean
    norm of row i of the round-up bound operand Abar (c_j: column j of Bbar),
    and e_i follows the rule of R3.  Then
    2 sum_h |a'_ih||b'_hj| <= 2^(e_i + f_j + 1) sum_h Abar_ih Bbar_hj
                           <= 2^(e_i + f_j + 1) sqrt(r_i c_j) <= P - 1,
    which is condition (3).  Squares of Abar are multiples of 2^-18, so r_i is
    an exact integer multiple of 2^-18 (below 2^34 for k <= 2^18).
R14 Karatsuba-only moduli (the list of Section III-B, used as an ablation of
    the hybrid list): p_l from the greedy scan down from 513, every one with
    the Karatsuba split s = 16; residues follow R7, so p = 513 gives digits
    in [-16, 16] like the hybrid list's largest moduli.
R15 INT8 arm (the INT8-based Ozaki-II scheme of Section II, the paper's
    baseline): moduli from the Section II list (greedy scan down from 256),
    one INT8 operand per modulus (the residue itself, in [-128, 127] by R7)
    and one integer product per modulus, exact in INT32 for k <= 2^16 per
    chunk.  The scale exponents come from the same bound as the FP8 arm (the
    FP8 bound product in accurate mode, R13 in fast mode): any upper bound
    that gives condition (3) serves, and sharing it makes the two arms differ
    only in their moduli and residue products.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

# ---------------------------------------------------------------------------
# OCP FP8 E4M3FN (Section III-A: integers -16..16 are exact in this format)
# ---------------------------------------------------------------------------


def e4m3_decode(code: int) -> float:
    """Value of an E4M3FN byte: 1 sign, 4 exponent (bias 7), 3 mantissa bits;
    exponent field 0 is subnormal; S.1111.111 is NaN; no infinities."""
    sign = -1.0 if code & 0x80 else 1.0
    ex = (code >> 3) & 0xF
    man = code & 0x7
    if ex == 0xF and man == 0x7:
        return float("nan")
    if ex == 0:
        return sign * man * 2.0 ** -9
    return sign * (8 + man) * 2.0 ** (ex - 10)


#: all non-negative finite E4M3 values, ascending (codes 0x00..0x7E)
E4M3_NONNEG = np.array([e4m3_decode(c) for c in range(0x7F)], dtype=np.float64)
E4M3_MIN_POS = E4M3_NONNEG[1]          # 2^-9
E4M3_MAX = E4M3_NONNEG[-1]             # 448


def e4m3_encode_exact(v: np.ndarray) -> np.ndarray:
    """Byte code of values that are exactly E4M3-representable (0 -> +0x00)."""
    v = np.asarray(v, dtype=np.float64)
    mag = np.abs(v)
    idx = np.searchsorted(E4M3_NONNEG, mag)
    idx = np.minimum(idx, len(E4M3_NONNEG) - 1)
    if not np.all(E4M3_NONNEG[idx] == mag):
        raise ValueError("value not representable in E4M3")
    code = idx.astype(np.uint8)
    return np.where((v < 0) & (code != 0), code | 0x80, code).astype(np.uint8)


def round_up_e4m3(x: np.ndarray, nonzero: np.ndarray) -> np.ndarray:
    """Smallest E4M3 value >= the exact non-negative x (Section III-E cast).

    `x` holds the float64 value of the exact product |a| 2^(7-E); that product
    is exact whenever it is at least 2^-1022.  Below that it may have rounded
    (even to 0), but any such exact value is far under 2^-9, whose round-up is
    2^-9, so `nonzero` (a != 0) settles those entries.
    """
    idx = np.searchsorted(E4M3_NONNEG, x, side="left")
    out = E4M3_NONNEG[idx]
    return np.where(nonzero & (out < E4M3_MIN_POS), E4M3_MIN_POS, out)


# ---------------------------------------------------------------------------
# Moduli (Sections II, III-B, III-D)
# ---------------------------------------------------------------------------


def _greedy_coprime(candidates, count):
    chosen = []
    for c in candidates:
        if all(math.gcd(c, q) == 1 for q in chosen):
            chosen.append(c)
            if len(chosen) == count:
                break
    return chosen


def int8_moduli(N: int) -> list[int]:
    """Section II list: scan down from 256, keep integers coprime to all kept."""
    return _greedy_coprime(range(256, 1, -1), N)


def karatsuba_moduli(N: int) -> list[int]:
    """Section III-B list: the same greedy scan, starting at 513."""
    return _greedy_coprime(range(513, 1, -1), N)


def hybrid_moduli(N: int) -> list[tuple[int, str, int]]:
    """Section III-D list as (p, kind, s).

    Squares up to 33^2 come first in descending order, then the list goes on
    with integers in descending order from 513; every candidate is kept when
    it is coprime to all kept so far.  That is one greedy descending scan over
    {s^2 : 2 <= s <= 33} united with {2, ..., 513}.  Squares (p = s^2) use
    s = sqrt(p) and the modular-reduction split; the others use Karatsuba with
    s = 16.  Below 34 moduli the squares are exactly p_1..p_6.
    """
    cands = sorted({s * s for s in range(2, 34)} | set(range(2, 514)), reverse=True)
    out = []
    for p in _greedy_coprime(cands, N):
        r = math.isqrt(p)
        out.append((p, "square", r) if r * r == p else (p, "karatsuba", 16))
    if len(out) < N:
        raise ValueError("not enough moduli")
    return out


def moduli_table(N: int, moduli_set: str = "hybrid") -> list[tuple[int, str, int]]:
    """The N moduli as (p, kind, s): the hybrid list of Section III-D, the
    Karatsuba-only list of Section III-B (every modulus with s = 16, R14), or
    the INT8 list of Section II (kind "int8", no digit split, R15)."""
    if moduli_set == "hybrid":
        return hybrid_moduli(N)
    if moduli_set in ("karatsuba", "int8"):
        lst = karatsuba_moduli(N) if moduli_set == "karatsuba" else int8_moduli(N)
        out = [(p, "karatsuba", 16) if moduli_set == "karatsuba" else (p, "int8", 0)
               for p in lst]
        if len(out) < N:
            raise ValueError("not enough moduli")
        return out
    raise ValueError("moduli_set must be 'hybrid', 'karatsuba' or 'int8'")


def crt_weights(moduli: list[int]) -> tuple[int, list[int]]:
    """P and the weights w_l = q_l P / p_l with q_l P/p_l = 1 (mod p_l)  (eq. CRT)."""
    P = math.prod(moduli)
    w = []
    for p in moduli:
        Pl = P // p
        q = pow(Pl, -1, p)
        w.append(q * Pl)
    return P, w


def smod(x, p):
    """Symmetric remainder in [-floor(p/2), ceil(p/2) - 1] (reading R7).
    Works elementwise on int64 arrays, object arrays of Python ints, or ints."""
    h = p // 2
    return ((x + h) % p) - h


# ---------------------------------------------------------------------------
# Step 1: scaling (Section II eq. def:A'/def:B', Section III-E)
# ---------------------------------------------------------------------------


def ufp_exponents(X: np.ndarray, axis: int) -> np.ndarray:
    """E with ufp(max |x|) = 2^E along `axis` (0 for all-zero lines), so that
    mu' = 2^(7 - E) (eq. def:mu'nu').  Exact: frexp splits the float."""
    amax = np.max(np.abs(X), axis=axis) if X.shape[axis] > 0 else \
        np.zeros(X.shape[1 - axis])
    _, e = np.frexp(amax)                 # amax = f 2^e, f in [0.5, 1)
    return np.where(amax > 0, e - 1, 0).astype(np.int64)


def bound_operands(opA: np.ndarray, opB: np.ndarray, EA: np.ndarray, EB: np.ndarray):
    """Abar = RU_e4m3(mu' |A|),  Bbar = RU_e4m3(|B| nu')  (Section III-E, R1)."""
    xa = np.ldexp(np.abs(opA), (7 - EA)[:, None])
    xb = np.ldexp(np.abs(opB), (7 - EB)[None, :])
    return (round_up_e4m3(xa, opA != 0), round_up_e4m3(xb, opB != 0))


def exact_bound_product(Abar: np.ndarray, Bbar: np.ndarray) -> np.ndarray:
    """Abar Bbar scaled by 2^18, as exact integers in float64 (R4).

    Abar, Bbar are multiples of 2^-9 not above 256, so 2^9 Abar and 2^9 Bbar are
    integers below 2^18; each product is below 2^34 and any partial sum over
    k <= 2^18 stays below 2^53, so the float64 matmul is exact."""
    if Abar.shape[1] > 2 ** 18:
        raise ValueError("k too large for an exact float64 bound product")
    return np.ldexp(Abar, 9) @ np.ldexp(Bbar, 9)


def cauchy_schwarz_norms(Abar: np.ndarray, Bbar: np.ndarray):
    """Squared Euclidean norms, scaled by 2^18, of the rows of Abar and the
    columns of Bbar (fast mode, R13), as exact integers in float64.

    2^9 Abar is an integer of at most 2^17, its square at most 2^34, and a sum
    of k <= 2^18 such squares at most 2^52, so every partial sum is an exact
    integer whatever order numpy sums in."""
    if Abar.shape[1] > 2 ** 18:
        raise ValueError("k too large for exact float64 norms")
    r18 = (np.ldexp(Abar, 9) ** 2).sum(axis=1)
    c18 = (np.ldexp(Bbar, 9) ** 2).sum(axis=0)
    return r18, c18


def scale_exponent(r18: int, P: int) -> int:
    """Largest integer e with 2^(2e+1) r <= P - 1, where r = r18 / 2^18 (R3, R5).

    Zero r gives 0 (R6)."""
    r18 = int(r18)
    if r18 == 0:
        return 0
    lim = Fraction((P - 1) * 2 ** 18)

    def ok(e):
        return Fraction(r18) * Fraction(2) ** (2 * e + 1) <= lim

    e = ((P - 1).bit_length() + 18 - r18.bit_length() - 1) // 2
    while ok(e + 1):
        e += 1
    while not ok(e):
        e -= 1
    return e


def to_integers(op: np.ndarray, shift: np.ndarray, axis: int) -> np.ndarray:
    """trunc(x 2^shift) with the shift applied per row (axis=0 -> shift[i] on
    row i) or per column (axis=1), held exactly in float64 (eq. def:A')."""
    sh = shift[:, None] if axis == 0 else shift[None, :]
    return np.trunc(np.ldexp(op, sh))


# ---------------------------------------------------------------------------
# Step 2: residues, FP8 digits, exact products, CRT (Sections II, III-B..D)
# ---------------------------------------------------------------------------


def residues(Xint: np.ndarray, p: int) -> np.ndarray:
    """smod(X', p) as int64.  Entries below 2^53 in magnitude are exact int64
    values and use integer remainder; larger ones use fmod, which is exact
    for every float64."""
    small = np.abs(Xint) < 2.0 ** 53
    r = np.empty(Xint.shape, dtype=np.int64)
    r[small] = Xint[small].astype(np.int64) % p
    r[~small] = np.fmod(Xint[~small], p).astype(np.int64)
    return smod(r, p)


def digits_square(u: np.ndarray, s: int):
    """Split for p = s^2 (Section III-D): x1 = round(u/s) half away from zero
    (R8), x2 = u - s x1.  Returns (x1, x2)."""
    x1 = np.sign(u) * ((np.abs(u) + s // 2) // s)
    return x1, u - s * x1


def digits_karatsuba(u: np.ndarray, s: int = 16):
    """Split for the other moduli (Section III-B): x1 = sign(u) ceil(|u|/s),
    x2 = u - s x1, x3 = x1 + x2.  Returns (x1, x2, x3)."""
    x1 = np.sign(u) * (-((-np.abs(u)) // s))
    x2 = u - s * x1
    return x1, x2, x1 + x2


def digit_slices(u: np.ndarray, kind: str, s: int) -> list[np.ndarray]:
    """The slices stored for one modulus: 2 FP8 digit slices for squares, 3
    for Karatsuba (workflow steps 5-6 of Section IV-B), and for the INT8 arm
    the residue itself as one INT8 slice (Section II)."""
    if kind == "int8":
        return [u]
    return list(digits_square(u, s) if kind == "square" else digits_karatsuba(u, s))


def _exact_int_matmul(X: np.ndarray, Y: np.ndarray, chunk: int = 2 ** 16) -> np.ndarray:
    """X @ Y for small-integer matrices, exact: k is summed in chunks whose
    float64 partial sums stay integers below 2^53; chunks add in int64."""
    m, k = X.shape
    out = np.zeros((m, Y.shape[1]), dtype=np.int64)
    for h in range(0, k, chunk):
        out += (X[:, h:h + chunk].astype(np.float64) @
                Y[h:h + chunk, :].astype(np.float64)).astype(np.int64)
    return out


def residue_product(uA: np.ndarray, uB: np.ndarray, p: int) -> np.ndarray:
    """C'_l = smod(A'_l B'_l, p_l) computed directly from the residues
    (eq. CRTmatmul).  |u| <= 545, so chunks of 2^16 keep sums below 2^35."""
    return smod(_exact_int_matmul(uA, uB), p)


def residue_product_fp8(dA: list, dB: list, p: int, kind: str, s: int,
                        chunk: int = 2 ** 16) -> np.ndarray:
    """C'_l from the digit products, as the MMA path forms it.

    Squares (eq. 3matmult-notKaratsuba): s A1 B2 + s A2 B1 + A2 B2 (mod p).
    Karatsuba (eq. C'-Karatsuba): s^2 C1 + C2 + s (C3 - C1 - C2) (mod p).
    Each FP8 digit product over a chunk of k <= 2^16 is an integer of
    magnitude at most 2^24 (eq. error-free-FP8-matmult); chunks are reduced
    modulo p.  INT8 (Section II): the one product of the residues, whose sum
    over a chunk stays inside INT32 (|u| <= 128, 2^16 2^14 = 2^30)."""
    m, k = dA[0].shape
    acc = np.zeros((m, dB[0].shape[1]), dtype=np.int64)
    for h in range(0, max(k, 1), chunk):
        sl = slice(h, h + chunk)
        G = lambda x, y: (dA[x][:, sl].astype(np.float64) @
                          dB[y][sl, :].astype(np.float64)).astype(np.int64)
        if kind == "square":
            v = s * G(0, 1) + s * G(1, 0) + G(1, 1)
        elif kind == "int8":
            v = G(0, 0)
            if v.size and int(np.max(np.abs(v))) >= 2 ** 31:
                raise ArithmeticError("INT32 accumulation would overflow")
        else:
            c1, c2, c3 = G(0, 0), G(1, 1), G(2, 2)
            v = s * s * c1 + c2 + s * (c3 - c1 - c2)
        acc = smod(acc + smod(v, p), p)
    return acc


def crt_reconstruct(planes: list[np.ndarray], moduli: list[int]) -> np.ndarray:
    """C' = smod(sum_l w_l C'_l, P) (eq. CRT_finalreduction), as Python ints."""
    P, w = crt_weights(moduli)
    S = np.zeros(planes[0].shape, dtype=object)
    for wl, pl in zip(w, planes):
        S = S + wl * pl.astype(object)
    return smod(S, P)


# ---------------------------------------------------------------------------
# Step 3: inverse scaling (eq. inversescaling) and alpha/beta (R10)
# ---------------------------------------------------------------------------


def _rn_scaled(x: int, t: int) -> float:
    """RN-even(x 2^-t) for an integer x; CPython's int true division and
    int->float conversion are correctly rounded (subnormals included)."""
    if t >= 0:
        return x / (1 << t)
    try:
        return float(x << (-t))
    except OverflowError:
        return math.copysign(math.inf, x)


def inverse_scale(Cp: np.ndarray, sA: np.ndarray, sB: np.ndarray) -> np.ndarray:
    """Chat_ij = RN(C'_ij 2^-(sA_i + sB_j)) with mu_i = 2^sA_i, nu_j = 2^sB_j."""
    m, n = Cp.shape
    out = np.empty((m, n), dtype=np.float64)
    for i in range(m):
        for j in range(n):
            out[i, j] = _rn_scaled(int(Cp[i, j]), int(sA[i]) + int(sB[j]))
    return out


# ---------------------------------------------------------------------------
# The whole path on logical operands op(A) (m x k) and op(B) (k x n)
# ---------------------------------------------------------------------------


def scaling(opA: np.ndarray, opB: np.ndarray, num_moduli: int, mode: str = "accurate",
            moduli_set: str = "hybrid") -> dict:
    """Workflow steps 1-3 of Section IV-B: mu', nu', the round-up FP8 bound
    operands, the bound product's line maxima (accurate mode) or the bound
    operands' line norms (fast mode, R13) and the scale exponents.
    Returns a dict with EA, EB, Abar, Bbar, r18, c18, e, f, sA = log2(mu),
    sB = log2(nu), the zeroed operands A, B and the non-finite flags."""
    if mode not in ("accurate", "fast"):
        raise ValueError("mode must be 'accurate' or 'fast'")
    opA = np.asarray(opA, dtype=np.float64)
    opB = np.asarray(opB, dtype=np.float64)
    m, k = opA.shape
    n = opB.shape[1]
    mods = moduli_table(num_moduli, moduli_set)
    P = math.prod(p for p, _, _ in mods)

    # R9: non-finite rows / columns are flagged and quantized as zeros
    badA = ~np.all(np.isfinite(opA), axis=1) if k else np.zeros(m, bool)
    badB = ~np.all(np.isfinite(opB), axis=0) if k else np.zeros(n, bool)
    A = np.where(np.isfinite(opA), opA, 0.0)
    B = np.where(np.isfinite(opB), opB, 0.0)

    # workflow step 1: mu', nu' and the round-up FP8 bound operands
    EA = ufp_exponents(A, axis=1)
    EB = ufp_exponents(B, axis=0)
    Abar, Bbar = bound_operands(A, B, EA, EB)

    if mode == "fast":
        # fast mode: Cauchy-Schwarz norms in place of the bound product (R13)
        r18, c18 = cauchy_schwarz_norms(Abar, Bbar)
    else:
        # workflow steps 2-3: bound product, row/column maxima, scale exponents
        W18 = exact_bound_product(Abar, Bbar)
        r18 = W18.max(axis=1) if n else np.zeros(m)
        c18 = W18.max(axis=0) if m else np.zeros(n)
        del W18
    e = np.array([scale_exponent(v, P) for v in r18], dtype=np.int64)
    f = np.array([scale_exponent(v, P) for v in c18], dtype=np.int64)
    return dict(moduli=mods, P=P, A=A, B=B, badA=badA, badB=badB, EA=EA, EB=EB,
                Abar=Abar, Bbar=Bbar, r18=r18, c18=c18, e=e, f=f,
                sA=7 - EA + e, sB=7 - EB + f)


def line_bounds(opA: np.ndarray, opB: np.ndarray, rows, cols, mode: str = "accurate",
                log=None) -> dict:
    """Workflow steps 1-2 of Section IV-B for the rows `rows` of op(A) and the
    columns `cols` of op(B) only: mu', nu' of those lines and the bound that
    decides their scale exponents (accurate mode: the maximum of the bound
    product over ALL partner lines; fast mode: the line's own norm, R13).

    The definitions are those of scaling(); only the bound-product entries
    that reach the requested maxima are formed: Abar[rows] Bbar gives the row
    maxima r_i, Abar Bbar[:, cols] the column maxima c_j.  The bound operands
    of both sides are built in full, because every partner line enters a
    maximum.  The result does not depend on the number of moduli, so one call
    serves every N (scaling_from_bounds).  `log`, if given, is called with a
    short message after each step (for progress reports on large inputs)."""
    say = log or (lambda msg: None)
    if mode not in ("accurate", "fast"):
        raise ValueError("mode must be 'accurate' or 'fast'")
    opA = np.asarray(opA, dtype=np.float64)
    opB = np.asarray(opB, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    k = opA.shape[1]
    finA = np.isfinite(opA)
    finB = np.isfinite(opB)
    badA = ~np.all(finA[rows], axis=1) if k else np.zeros(len(rows), bool)
    badB = ~np.all(finB[:, cols], axis=0) if k else np.zeros(len(cols), bool)
    A = np.where(finA, opA, 0.0)
    B = np.where(finB, opB, 0.0)
    del finA, finB
    EA = ufp_exponents(A, axis=1)
    EB = ufp_exponents(B, axis=0)
    Abar, Bbar = bound_operands(A, B, EA, EB)
    say("bound operands")
    if mode == "fast":
        r18, c18 = cauchy_schwarz_norms(Abar[rows], Bbar[:, cols])
    else:
        n, m = B.shape[1], A.shape[0]
        r18 = exact_bound_product(Abar[rows], Bbar).max(axis=1) if n else np.zeros(len(rows))
        say("row maxima")
        c18 = exact_bound_product(Abar, Bbar[:, cols]).max(axis=0) if m else np.zeros(len(cols))
        say("column maxima")
    return dict(A=A[rows], B=B[:, cols], badA=badA, badB=badB, EA=EA[rows], EB=EB[cols],
                r18=r18, c18=c18, mode=mode)


def scaling_from_bounds(bounds: dict, num_moduli: int, moduli_set: str = "hybrid") -> dict:
    """Step 3 (the scale exponents, Section III-E, R3) for the lines of
    line_bounds(); returns a scaling dict of the sub-problem
    op(A)[rows] x op(B)[:, cols] whose lines carry the exponents of the whole
    problem, so products(sc, slice(None), slice(None)) yields the sampled
    outputs Chat[rows][:, cols]."""
    mods = moduli_table(num_moduli, moduli_set)
    P = math.prod(p for p, _, _ in mods)
    e = np.array([scale_exponent(v, P) for v in bounds["r18"]], dtype=np.int64)
    f = np.array([scale_exponent(v, P) for v in bounds["c18"]], dtype=np.int64)
    sc = {key: bounds[key] for key in ("A", "B", "badA", "badB", "EA", "EB", "r18", "c18")}
    sc.update(moduli=mods, P=P, e=e, f=f, sA=7 - bounds["EA"] + e, sB=7 - bounds["EB"] + f)
    return sc


def scaling_lines(opA: np.ndarray, opB: np.ndarray, num_moduli: int, rows, cols,
                  mode: str = "accurate", moduli_set: str = "hybrid") -> dict:
    """scaling() restricted to the rows `rows` and columns `cols` (see
    line_bounds and scaling_from_bounds)."""
    return scaling_from_bounds(line_bounds(opA, opB, rows, cols, mode), num_moduli, moduli_set)


def products(sc: dict, rows, cols, keep_stages: bool = False):
    """Workflow steps 4-10 for the entries (rows x cols): integers, residues,
    exact residue products, CRT and inverse scaling."""
    A = sc["A"][rows]
    B = sc["B"][:, cols]
    sA = sc["sA"][rows]
    sB = sc["sB"][cols]
    # workflow steps 4-6: integers, residues, digits
    Aint = to_integers(A, sA, axis=0)
    Bint = to_integers(B, sB, axis=1)
    planes, per_mod = [], []
    for p, kind, s in sc["moduli"]:
        uA = residues(Aint, p)
        uB = residues(Bint, p)
        # workflow steps 7-8: the residue product, exact (eq. CRTmatmul)
        planes.append(residue_product(uA, uB, p))
        if keep_stages:
            per_mod.append(dict(p=p, kind=kind, s=s, uA=uA, uB=uB,
                                dA=digit_slices(uA, kind, s),
                                dB=digit_slices(uB, kind, s)))
    # workflow steps 9-10: CRT and inverse scaling
    Cp = crt_reconstruct(planes, [p for p, _, _ in sc["moduli"]])
    Chat = inverse_scale(Cp, sA, sB)
    Chat[sc["badA"][rows], :] = np.nan
    Chat[:, sc["badB"][cols]] = np.nan
    return Chat, dict(Aint=Aint, Bint=Bint, planes=planes, per_modulus=per_mod, Cp=Cp)


def emulate(opA: np.ndarray, opB: np.ndarray, num_moduli: int,
            keep_stages: bool = False, mode: str = "accurate", moduli_set: str = "hybrid"):
    """Chat ~ op(A) op(B) by the FP8 Ozaki-II scheme, accurate or fast mode.

    Returns Chat (m x n float64) and, with keep_stages, a dict of every
    intermediate quantity.  Implements Sections II and III-B..III-E in the
    order of the workflow of Section IV-B."""
    sc = scaling(opA, opB, num_moduli, mode, moduli_set)
    m, n = sc["A"].shape[0], sc["B"].shape[1]
    Chat, st = products(sc, slice(0, m), slice(0, n), keep_stages)
    if not keep_stages:
        return Chat
    st.update({key: sc[key] for key in ("moduli", "P", "EA", "EB", "Abar", "Bbar", "r18",
                                        "c18", "e", "f", "sA", "sB", "badA", "badB")})
    return Chat, st


def emulate_sampled(opA: np.ndarray, opB: np.ndarray, num_moduli: int, rows, cols,
                    mode: str = "accurate", moduli_set: str = "hybrid"):
    """The entries Chat[rows][:, cols] of emulate(opA, opB, num_moduli), with
    the scale exponents of every line (they depend on the whole product) but
    the residue products, CRT and inverse scaling only for the sample.
    Returns (Chat_sample, scaling dict)."""
    sc = scaling(opA, opB, num_moduli, mode, moduli_set)
    Chat, _ = products(sc, np.asarray(rows), np.asarray(cols), False)
    return Chat, sc


def combine_alpha_beta(Chat: np.ndarray, alpha: float, beta: float,
                       Cin: np.ndarray | None) -> np.ndarray:
    """C = RN(alpha Chat) when beta == 0 (C_in unread), else
    RN(RN(alpha Chat) + RN(beta C_in))  (R10)."""
    t = np.float64(alpha) * Chat
    if beta == 0.0:
        return t
    return t + np.float64(beta) * Cin


# ---------------------------------------------------------------------------
# BLAS-style entry point (column-major storage, transA/transB)
# ---------------------------------------------------------------------------


def _op_view(buf, trans, rows, cols, ld):
    """Logical op(X) (rows x cols) out of a flat column-major buffer."""
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    if rows == 0 or cols == 0:
        return np.zeros((rows, cols))
    if trans in "Nn":
        return np.lib.stride_tricks.as_strided(buf, (rows, cols), (8, 8 * ld)).copy()
    return np.lib.stride_tricks.as_strided(buf, (rows, cols), (8 * ld, 8)).copy()


def dgemm(transA: str, transB: str, m: int, n: int, k: int, alpha: float,
          A: np.ndarray, lda: int, B: np.ndarray, ldb: int, beta: float,
          C: np.ndarray, ldc: int, num_moduli: int, mode: str = "accurate",
          moduli_set: str = "hybrid") -> np.ndarray:
    """Column-major C <- alpha op(A) op(B) + beta C, emulated; returns a new
    flat C buffer (entries outside the m x n view are copied unchanged)."""
    Cout = np.array(C, dtype=np.float64, copy=True)
    if m == 0 or n == 0:
        return Cout
    view = np.lib.stride_tricks.as_strided(Cout, (m, n), (8, 8 * ldc))
    Cin = view.copy()
    if k == 0 or alpha == 0.0:
        view[...] = 0.0 if beta == 0.0 else np.float64(beta) * Cin
        return Cout
    opA = _op_view(A, transA, m, k, lda)
    opB = _op_view(B, transB, k, n, ldb)
    Chat = emulate(opA, opB, num_moduli, mode=mode, moduli_set=moduli_set)
    view[...] = combine_alpha_beta(Chat, alpha, beta, Cin)
    return Cout
