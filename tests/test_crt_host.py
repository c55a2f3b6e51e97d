"""The library's CRT arithmetic (eq. CRT_finalreduction and the one rounding
of eq. inversescaling, the header the CRT kernel uses), compiled for the host
with the library's own tables, against exact integer results: for residues
u_l = C mod p_l the reconstruction must return RN(C 2^-t) bit for bit, for C
anywhere in the symmetric range [-floor(P/2), P - 1 - floor(P/2)].  Cases
cover both ends of the range, the edge of the kernel's fast range check
(2^-40 P below P/2), zero, rounding ties, subnormal and overflowing results,
and every limb count of P (N = 1..33)."""
import math
import os
import random
import shutil
import struct
import subprocess

import pytest

from oracle import ozaki2_ref as ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_10634_amd", "csrc")
LISTS = {"hybrid": 0, "karatsuba": 1, "int8": 2}


# Host builds of the checker: hipcc (the compiler of the library), and g++
# with AddressSanitizer and UndefinedBehaviorSanitizer (any finding aborts).
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module", params=["hipcc", "sanitized"])
def checker(request, tmp_path_factory):
    out = str(tmp_path_factory.mktemp("crt") / f"crt_host_check_{request.param}")
    srcs = [os.path.join(ROOT, "tests", "crt_host_check.cpp"), os.path.join(CSRC, "oz2_tables.cpp")]
    flags = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC]
    if request.param == "hipcc":
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available")
        cmd = [hipcc, "-O2", *flags, "-x", "c++", *srcs, "-o", out]
    else:
        gxx = shutil.which("g++")
        if not gxx:
            pytest.skip("g++ not available")
        cmd = [gxx, "-O1", "-g", *SANITIZE, *flags, *srcs, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _smod(x, P):
    h = P // 2
    return (x + h) % P - h


def _rn(x, t):
    """RN-even(x 2^-t): Python's int true division and int -> float conversion
    round correctly (subnormals included)."""
    if t >= 0:
        return x / (1 << t)
    try:
        return float(x << -t)
    except OverflowError:
        return math.copysign(math.inf, x)


def _bits(v):
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def _targets(P, rng, count):
    h = P // 2
    out = [0, 1, -1, 2, -2, h, -h, P - 1 - h, h - 1, -h + 1]
    for d in range(1, 4):
        out += [h - d, -h + d, P - 1 - h - d]
    for e in (39, 40, 41):
        edge = h - (P >> e)
        out += [edge + d for d in range(-2, 3)] + [-(edge + d) for d in range(-2, 3)]
    # leading bits at and next to the 32-bit limb boundaries, with the bits
    # below the 53 kept ones a tie, a tie plus one, or a round bit and one far
    # sticky bit
    for bl in (31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 129):
        if bl >= P.bit_length():
            continue
        top = rng.getrandbits(53) | (1 << 52)
        k = bl - 53
        if k < 2:
            out.append(top << max(k, 0))
            continue
        tie = (top << k) | (1 << (k - 1))
        out += [tie, -tie, tie + 1, tie - 1, tie | 1]
    for _ in range(count):
        r = rng.random()
        if r < 0.4:
            c = rng.randrange(-h, P - h)
        elif r < 0.7:
            c = rng.choice([-1, 1]) * rng.getrandbits(rng.randrange(1, P.bit_length()))
        else:
            k = rng.randrange(0, max(1, P.bit_length() - 56))
            c = (rng.getrandbits(54) | 1) << k
            c += rng.choice([0, 1, 1 << max(k - 1, 0), (1 << max(k - 1, 0)) - 1])
            c *= rng.choice([-1, 1])
        out.append(c)
    return [_smod(c, P) for c in out]


def _shift(c, P, rng):
    r = rng.random()
    if r < 0.5:
        return P.bit_length() - 53 + rng.randrange(-60, 60)
    if r < 0.8:
        return rng.randrange(-1100, 1300)
    return 1074 + max(abs(c), 1).bit_length() + rng.randrange(-60, 3)


@pytest.mark.parametrize("moduli", ["hybrid", "karatsuba", "int8"])
def test_crt_reconstruction_exact(checker, moduli):
    rng = random.Random(8100 + LISTS[moduli])
    Ns = range(1, 34) if moduli == "hybrid" else (1, 2, 5, 13, 14, 16, 20, 33)
    for N in Ns:
        mods = [p for p, _, _ in ref.moduli_table(N, moduli)]
        P = math.prod(mods)
        lines, want = [], []
        for c in _targets(P, rng, 200):
            us = []
            for p in mods:
                u = c % p
                us.append(u - p if u > p - 1 - p // 2 else u)
            t = _shift(c, P, rng)
            lines.append(" ".join(str(v) for v in [t] + us))
            want.append(_bits(_rn(c, t)))
        res = subprocess.run([checker, str(N), str(LISTS[moduli])], input="\n".join(lines) + "\n",
                             capture_output=True, text=True, check=True)
        got = [int(x, 16) for x in res.stdout.split()]
        assert len(got) == len(want), (moduli, N)
        bad = [(ln, hex(g), hex(w)) for ln, g, w in zip(lines, got, want) if g != w]
        assert not bad, (moduli, N, bad[:3])
