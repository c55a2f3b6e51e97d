"""The accurate mode's decision window (oz2_window.h, compiled for the host
with the library's tables) against a host model of the FP8 MFMA's
accumulation under the stated worst case (W) the window is derived from:
inside each group of 8 consecutive k every product but the group's largest
may move by up to 2^-13 ufp(largest), either way; every addition of a group
sum into the FP32 accumulator may round by up to one ulp, either way.

For adversarial non-negative patterns (one large product per group with
seven just below the truncation grid; sums whose every addition loses almost
an ulp; wide exponent spreads; random E4M3 products), k from 64 to 2^18, the
k range summed whole or in 16 parts whose sums are then added (the split
bound product), and the extreme choices of the model (every deviation down,
every deviation up, and the measured hardware's truncation), the exact line
maximum must lie in the library's window, and a line the window settles must get the exponent
of its exact maximum (the oracle's rule, Section III-E)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ozaki2_ref as ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_10634_amd", "csrc")

KS = [64, 256, 1024, 4096, 16384, 65536, 1 << 18]
E4M3 = ref.E4M3_NONNEG[1:]          # positive finite E4M3 values


# Host builds of the window: hipcc (the compiler of the library), and g++ with
# AddressSanitizer and UndefinedBehaviorSanitizer (any finding aborts).
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module", params=["hipcc", "sanitized"])
def window(request, tmp_path_factory):
    out = str(tmp_path_factory.mktemp("window") / f"window_host_check_{request.param}")
    srcs = [os.path.join(ROOT, "tests", "window_host_check.cpp"),
            os.path.join(CSRC, "oz2_tables.cpp")]
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

    def call(N, pairs, parts=1):
        text = "".join(f"{kp} {parts} {int(b):08x}\n" for kp, b in pairs)
        r = subprocess.run([out, str(N), "0"], input=text, capture_output=True, text=True,
                           check=True)
        rows = [ln.split() for ln in r.stdout.splitlines()]
        return [(float.fromhex(a), float.fromhex(b), int(c), int(d)) for a, b, c, d in rows]

    return call


def _round_f32(v, direction):
    """v (float64 array) rounded to FP32 toward -inf (direction < 0), +inf
    (> 0) or to nearest (0): each within one ulp of v."""
    f = v.astype(np.float32)
    if direction < 0:
        f = np.where(f.astype(np.float64) > v, np.nextafter(f, np.float32(-np.inf)), f)
    elif direction > 0:
        f = np.where(f.astype(np.float64) < v, np.nextafter(f, np.float32(np.inf)), f)
    return f


def mfma_model(x, how, parts=1):
    """Computed sums of the rows of x (non-negative products, k a multiple
    of 8) under (W): how = "down" (every product and addition deviates
    down), "up" (every one up) or "hw" (the measured behaviour: products
    truncated toward zero to the group's grid, additions truncated).  With
    parts > 1 the k range is cut into that many ranges of whole 256-blocks
    (as the split bound product does), each summed so, and the partial sums
    are then added in order with the same rounding direction."""
    if parts > 1:
        nb = x.shape[1] // 256
        cuts = [q * nb // parts * 256 for q in range(parts + 1)]
        direction = 1 if how == "up" else -1
        t = mfma_model(x[:, cuts[0]:cuts[1]], how)
        for q in range(1, parts):
            t = _round_f32(t.astype(np.float64) + mfma_model(x[:, cuts[q]:cuts[q + 1]], how),
                           direction)
        return t
    E, k = x.shape
    g = x.reshape(E, k // 8, 8)
    gmax = g.max(axis=2)
    ufp = np.where(gmax > 0, np.exp2(np.floor(np.log2(np.where(gmax > 0, gmax, 1.0)))), 0.0)
    grid = ufp * 2.0 ** -13
    first = np.zeros(g.shape, bool)
    np.put_along_axis(first, g.argmax(axis=2)[..., None], True, axis=2)
    step = grid[..., None] * (1.0 - 2.0 ** -30)
    if how == "down":
        gt = np.where(first, g, g - step)
    elif how == "up":
        gt = np.where(first, g, g + step)
    else:
        gt = np.where(first, g, np.floor(g / np.where(grid > 0, grid, 1.0)[..., None])
                      * grid[..., None])
    s = gt.sum(axis=2)
    direction = 1 if how == "up" else -1
    t = np.zeros(E, np.float32)
    for q in range(s.shape[1]):
        t = _round_f32(t.astype(np.float64) + s[:, q], direction)
    return t


def _exact18(x):
    """2^18 x the exact row sums (products of E4M3 values are multiples of 2^-18)."""
    return np.rint(np.ldexp(x, 18)).astype(np.int64).sum(axis=1)


def _pattern(kind, k, rng):
    """Products x[j, h] = Abar_ih Bbar_hj >= 0 of one line i against 6 partner
    lines j, every factor an E4M3 value."""
    E = 6
    if kind == "dominant":
        # per group one 256 x 256 and seven products just below its 2^-13 grid (8)
        a = np.full(k, 2.75)
        a[::8] = 256.0
        b = np.full((E, k), 2.75)
        b[:, ::8] = 256.0
        x = a[None, :] * b                      # 7.5625 < 8 = the grid
    elif kind == "ulp_loss":
        # one large first group, then small sums with awkward mantissas that
        # fall below the accumulator's ulp on every addition
        a = rng.choice(E4M3[(E4M3 >= 1.0) & (E4M3 <= 2.0)], size=k)
        b = rng.choice(E4M3[(E4M3 >= 1.0) & (E4M3 <= 2.0)], size=(E, k))
        a[:8] = 256.0
        b[:, :8] = 256.0
        x = a[None, :] * b
    elif kind == "spread":
        a = rng.choice(E4M3, size=k)
        b = rng.choice(E4M3, size=(E, k))
        x = a[None, :] * b
    else:  # "uniform": scaled inputs in [128, 256] per line, the usual case
        a = rng.choice(E4M3[E4M3 >= 16.0], size=k)
        b = rng.choice(E4M3[E4M3 >= 16.0], size=(E, k))
        x = a[None, :] * b
    # near-ties: a partner slightly below the largest, so the maximum of the
    # computed values may come from another line than the exact maximum
    x[1] = x[0]
    x[1, -1] = 0.0
    return x


@pytest.mark.parametrize("parts", [1, 16])
@pytest.mark.parametrize("kind", ["dominant", "ulp_loss", "spread", "uniform"])
def test_window_holds_exact_maximum(window, kind, parts):
    rng = np.random.default_rng(4242)
    P = ref.crt_weights([p for p, _, _ in ref.moduli_table(12)])[0]
    cases = []
    for k in KS:
        if k < 256 * parts:
            continue
        x = _pattern(kind, k, rng)
        r18 = int(_exact18(x).max())
        for how in ("down", "up", "hw"):
            rp = float(mfma_model(x, how, parts).max())
            cases.append((k, how, r18, rp))
    out = window(12, [(k, np.float32(rp).view(np.uint32)) for k, _, _, rp in cases], parts)
    for (k, how, r18, rp), (lo, hi, es, el) in zip(cases, out):
        r = float(r18) * 2.0 ** -18            # exact: r18 < 2^53
        assert lo <= r <= hi, (kind, k, how, r, rp, lo, hi)
        # a settled line gets the exponent of its exact maximum
        if es == el:
            assert es == ref.scale_exponent(r18, P), (kind, k, how)
        # the window is twice the deviation of (W), not more: it bounds the
        # share of lines that need the exact fix-up
        Q = k // 8 + parts - 1
        width = 2 * (7 * 2.0 ** -13 + 1.02 * Q * 2.0 ** -23) + 2 * (7 * 2.0 ** -13 + Q * 2.0 ** -23)
        assert hi / lo - 1 <= 1.01 * width


def test_window_settles_only_exact_exponents(window):
    # r' swept across scale thresholds: whenever both ends of the window give
    # one exponent, every value inside the window has it too
    P = ref.crt_weights([p for p, _, _ in ref.moduli_table(12)])[0]
    D = float(P - 1)
    rng = np.random.default_rng(11)
    pairs, rs = [], []
    for k in KS:
        for e in range(38, 67, 2):
            thr = D / 2.0 ** (2 * e + 1)     # a threshold of the rule (r in [2^-18, 2^35])
            for f in rng.uniform(0.99, 1.01, 40):
                rp = np.float32(thr * f)
                pairs.append((k, rp.view(np.uint32)))
                rs.append(float(rp))
    out = window(12, pairs)
    settled = 0
    for (k, _), rp, (lo, hi, es, el) in zip(pairs, rs, out):
        assert lo < rp < hi
        assert es <= el
        if es == el:
            settled += 1
            for v in np.linspace(lo, hi, 7):
                r18 = int(np.floor(v * 2.0 ** 18))
                if r18 > 0 and lo <= r18 * 2.0 ** -18:
                    assert ref.scale_exponent(r18, P) == es
    assert settled > len(pairs) // 2
