"""Parity of the HIP path with the CPU oracle, through the C ABI.

Every stage the library stores (exponents, FP8 bound operands, FP8 digit
slices, int16 residue planes) and the final C are compared bit for bit with
the oracle on seeded inputs whose sizes span several tiles and leave ragged
tails; the full-size workload is checked on sampled outputs."""
import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import phi_matrix, integer_matrix, normal_matrix, config_seed
from workloads.reference import dd_dot_rows, normalised_error

from gpu_util import run, check_stages, split

pytestmark = pytest.mark.gpu


def _inputs(m, n, k, phi, seed):
    if phi is None:
        return normal_matrix(m, k, seed), normal_matrix(k, n, seed + 1)
    return phi_matrix(m, k, phi, seed), phi_matrix(k, n, phi, seed + 1)


def _same(a, b):
    """Bit-identical float64 arrays (NaN payloads aside)."""
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


@pytest.mark.parametrize("N", [1, 2, 3, 6, 7, 12, 13, 20, 26, 33])
def test_stage_parity_ragged(N):
    print(f"stage parity N={N} shape=(300, 200, 700)", flush=True)
    A, B = _inputs(300, 200, 700, 1.0, 1000 + N)
    r = run(A, B, N, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, N, keep_stages=True)
    check_stages(r, A, B, N, st)
    assert _same(r.C, Chat)


@pytest.mark.parametrize("phi", [None, 0.5, 2.0, 4.0, 6.0])
@pytest.mark.parametrize("shape", [(256, 256, 256), (129, 385, 200), (64, 64, 1),
                                   (1, 300, 513), (520, 1, 77)])
def test_parity_shapes(phi, shape):
    m, n, k = shape
    print(f"parity shape={shape} phi={phi}", flush=True)
    A, B = _inputs(m, n, k, phi, 2000 + m + n + k)
    r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    check_stages(r, A, B, 12, st)
    assert _same(r.C, Chat)


def test_row_major_config_256():
    # 256^3 row-major, entries (U-0.5) exp(0.5 N(0,1)), alpha 1, beta 0, N = 12
    s = config_seed(1)
    A = phi_matrix(256, 256, 0.5, s)
    B = phi_matrix(256, 256, 0.5, s + 1)
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    C = oz.dgemm(tA, tB, 12)
    torch.cuda.synchronize()
    assert _same(C.cpu().numpy(), ref.emulate(A, B, 12))


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T"),
                                   ("t", "c"), ("C", "n")])
def test_transposes(ta, tb):
    print(f"transposes {ta}{tb}", flush=True)
    A, B = _inputs(190, 260, 333, 1.0, 3000)
    want = ref.emulate(A, B, 12)
    r = run(A, B, 12, transA=ta, transB=tb, pad=(3, 5, 2))
    assert r.status == 0
    assert _same(r.C, want)
    # entries of C outside the m x n view are untouched
    Cb = r.Cbuf.reshape(-1, r.ldc)
    assert np.all(Cb[:, r.m:] == 7.0)


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-2.5, 0.0), (0.75, 1.0), (1.0, -0.5),
                                        (0.0, 3.0), (0.0, 0.0)])
def test_alpha_beta(alpha, beta):
    A, B = _inputs(100, 90, 150, 1.0, 4000)
    Cin = phi_matrix(100, 90, 1.0, 4002)
    r = run(A, B, 12, alpha=alpha, beta=beta, Cin=Cin, pad=(0, 0, 4))
    assert r.status == 0
    if alpha == 0.0:
        want = np.zeros_like(Cin) if beta == 0.0 else beta * Cin
    else:
        want = ref.combine_alpha_beta(ref.emulate(A, B, 12), alpha, beta, Cin)
    assert _same(r.C, want)


def test_alpha_beta_cancellation_rounds_twice():
    """alpha Chat + beta C_in with heavy cancellation: the result must be
    RN(RN(alpha Chat) + RN(beta C_in)), two roundings, not one fused
    multiply-add (which differs exactly when the two terms cancel)."""
    A, B = _inputs(130, 70, 200, 1.0, 4200)
    Chat = ref.emulate(A, B, 12)
    noise = phi_matrix(130, 70, 1.0, 4201) * 1e-9
    alpha, beta = 2.0, -1.5
    Cin = (alpha / -beta) * Chat * (1.0 + noise)        # beta C_in ~ -alpha Chat
    r = run(A, B, 12, alpha=alpha, beta=beta, Cin=Cin, pad=(0, 0, 3))
    assert r.status == 0
    want = ref.combine_alpha_beta(Chat, alpha, beta, Cin)
    assert _same(r.C, want)


def test_beta_zero_does_not_read_C():
    A, B = _inputs(70, 50, 40, 1.0, 4100)
    Cin = np.full((70, 50), np.nan)
    r = run(A, B, 12, Cin=Cin)
    assert r.status == 0 and not np.any(np.isnan(r.C))


def test_zero_lines_and_nonfinite():
    A, B = _inputs(150, 140, 90, 1.0, 5000)
    A[3, :] = 0.0
    B[:, 7] = 0.0
    A[10, 5] = np.inf
    A[11, 0] = -np.inf
    B[20, 9] = np.nan
    r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    assert _same(r.C, Chat)
    assert np.all(np.isnan(r.C[10])) and np.all(np.isnan(r.C[:, 9]))
    assert np.all(r.C[3, :9] == 0) and not np.signbit(r.C[3, :9]).any()
    check_stages(r, A, B, 12, st)


def test_subnormal_and_extreme_magnitudes():
    A, B = _inputs(96, 80, 120, 1.0, 5100)
    A[0] *= 2.0 ** -1060           # row of subnormals and tiny normals
    A[1, :] = 0.0
    A[1, 3] = 5e-324               # a lone smallest subnormal
    A[2] *= 2.0 ** 900             # huge row
    B[:, 0] *= 2.0 ** -1000
    B[:, 1] *= 2.0 ** 1000
    r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    check_stages(r, A, B, 12, st)
    assert _same(r.C, Chat)


def test_integer_inputs_give_exact_product():
    A = integer_matrix(200, 300, 1000, 5200)
    B = integer_matrix(300, 150, 1000, 5201)
    r = run(A, B, 12)
    assert r.status == 0
    assert np.array_equal(r.C, A @ B)      # |sums| < 2^53: the float64 matmul is exact


@pytest.mark.parametrize("k,parts", [(32768, 0), (40000, 0), (65536, 0), (65536 + 300, 0),
                                     (65536 + 300, 4), (1 << 18, 0)])
def test_long_k_chunks(k, parts):
    # every k part of the residue products is at most 2^15 long (so at least
    # ceil(k / 2^15) parts), each in its own copy of the planes that the CRT
    # sums: the rule's 8 parts for this small output, a forced 4, and 8
    # parts of exactly 2^15 at the largest supported k
    print(f"long k={k} parts={parts}", flush=True)
    A, B = _inputs(40, 72, k, 1.0, 6000 + k)
    with split(parts):
        r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    P = r.planes(12, [pm["p"] for pm in st["per_modulus"]])
    for l, plane in enumerate(st["planes"]):
        assert np.array_equal(P[l, :72, :40].T.astype(np.int64), plane), f"plane {l}"
    assert _same(r.C, Chat)


def test_exact_fixups_many_lines_both_sides():
    # rows of op(A) with n_i leading ones and columns of op(B) with n'_j
    # leading ones: (Abar Bbar)_ij = 2^14 min(n_i, n'_j), so r_i = 2^14 n_i
    # and c_j = 2^14 n'_j, spread over 64 consecutive counts around a
    # threshold of the exponent rule.  The FP32 maxima are exact, yet every
    # line within the window's width of the threshold (several dozen, on both
    # sides, in groups of mixed sides) goes to the exact fix-up; k = 8448
    # also leaves a 256-k tail of the fix-up's 512-k chunks and splits the
    # bound product in 2 parts.
    k, N = 8448, 12
    P = ref.crt_weights([p for p, _, _ in ref.moduli_table(N)])[0]
    # threshold r = (P - 1) / 2^(2e+1) with r / 2^14 in [2^11, 2^13)
    e = ((P - 1).bit_length() - 1 - 14 - 13) // 2
    nstar = (P - 1) / 2.0 ** (2 * e + 1) / 2.0 ** 14
    assert 2 ** 11 <= nstar < 2 ** 13 - 64
    counts = int(nstar) - 32 + np.arange(64)
    A = (np.arange(k)[None, :] < counts[:, None]).astype(np.float64)
    B = A.T.copy()
    Chat, st = ref.emulate(A, B, N, keep_stages=True)
    assert len(set(st["e"].tolist())) == 2 and len(set(st["f"].tolist())) == 2
    r = run(A, B, N, keep_ws=True)
    assert r.status == 0
    print(f"many fix-ups: {r.fixups()} lines", flush=True)
    assert r.fixups() >= 20
    check_stages(r, A, B, N, st)
    assert _same(r.C, Chat)
    assert np.array_equal(r.C, np.minimum(counts[:, None], counts[None, :]).astype(np.float64))


def _constant_case(k):
    """Constant op(A) = c 2^-7 and op(B) = d 2^-7 (c, d in [128, 256)) chosen
    so that some digit product is 16 x 16: every FP8 product sum of that
    modulus then reaches 256 k, the exactness limit's order at k = 2^15."""
    for c in range(128, 256):
        for d in (c, 255, 200, 129):
            A = np.full((1, k), c / 128.0)
            B = np.full((k, 1), d / 128.0)
            _, st = ref.emulate(A, B, 12, keep_stages=True)
            for pm in st["per_modulus"]:
                pairs = ([(0, 1), (1, 0), (1, 1)] if pm["kind"] == "square"
                         else [(0, 0), (1, 1), (2, 2)])
                for x, y in pairs:
                    if abs(int(pm["dA"][x][0, 0]) * int(pm["dB"][y][0, 0])) == 256:
                        return c / 128.0, d / 128.0
    raise AssertionError("no extreme-digit constant found")


def test_extreme_digit_sums_exact():
    # product sums of 256 k = 2^23 per FP8 product at k = 2^15 must be exact
    # (one k part: a single accumulation over all 2^15)
    k = 32768
    a, b = _constant_case(k)
    A = np.full((64, k), a)
    B = np.full((k, 96), b)
    A[1::2] *= -1.0
    with split(1):
        r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    check_stages(r, A, B, 12, st)
    assert _same(r.C, Chat)


def _square_extreme_value(shift, base=1.0625, target=544, p=1089):
    """A value v in (1, 1.125] (so its round-up FP8 bound, and with it the
    scale shift, stays that of `base`) whose scaled integer trunc(v 2^shift)
    is congruent to `target` modulo p."""
    g = max(int(shift) - 52, 0)
    t0 = int(base * 2.0 ** (int(shift) - g))
    t = t0 - t0 % p + target * pow(2 ** g, -1, p) % p
    if t < t0:
        t += p
    return float(np.ldexp(float(t), g - int(shift)))


def test_square_cross_sums_reach_2_24():
    # Residues 544 = 16 * 33 + 16 modulo 1089 on both sides give the square
    # digits (16, 16), so A1 B2 + A2 B1 = 512 per k: over k = 2^15 the square
    # kernel's first two passes sum to exactly +-2^24 in FP32 (rows of both
    # signs), then fold and add A2 B2 = 256 k.
    k = 32768
    one = np.full((1, k), 1.0625)
    sc = ref.scaling(one, one.T.copy(), 12)
    v = _square_extreme_value(sc["sA"][0])
    w = _square_extreme_value(sc["sB"][0])
    A = np.full((64, k), v)
    B = np.full((k, 96), w)
    A[1::2] *= -1.0
    print(f"square cross sums k={k} v={v!r} w={w!r}", flush=True)
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    pm = next(q for q in st["per_modulus"] if q["p"] == 1089)
    a1, a2 = int(pm["dA"][0][0, 0]), int(pm["dA"][1][0, 0])
    b1, b2 = int(pm["dB"][0][0, 0]), int(pm["dB"][1][0, 0])
    assert (a1, a2, b1, b2) == (16, 16, 16, 16)
    assert (int(pm["dA"][0][1, 0]), int(pm["dA"][1][1, 0])) == (-16, -16)
    with split(1):   # one k part: a single accumulation over all 2^15
        r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    check_stages(r, A, B, 12, st)
    assert _same(r.C, Chat)


def _bound_case(kind):
    if kind == "spread":
        return _inputs(300, 280, 1000, 2.0, 7000)
    if kind == "split":
        # one output tile, k = 20000: the bound product runs as 4 k parts
        return _inputs(200, 190, 20000, 2.0, 7003)
    if kind == "wide":
        return _inputs(256, 256, 4096, 4.0, 7001)
    # one dominant entry per 64-block and many small ones with awkward
    # mantissas: the pattern that loses the most to truncating accumulation
    rng = np.random.default_rng(7002)
    A = rng.uniform(1.0, 2.0, (128, 2048)) * 2.0 ** -7
    A[:, ::64] = 1.0
    B = rng.uniform(1.0, 2.0, (2048, 128))
    return A, B


def _bound_parts(m, n, kp):
    """k parts of a single call's bound product (fewer than 128 output tiles
    and k of at least 8192: up to 16 parts of at least 4096, about 256
    workgroups)."""
    tiles = -(-m // 256) * -(-n // 256)
    if tiles >= 128 or kp < 8192:
        return 1
    return min(-(-256 // tiles), kp // 4096, 16)


@pytest.mark.parametrize("kind", ["spread", "wide", "dominant", "split"])
def test_bound_maxima_within_window(kind):
    # the GPU's FP32 line maxima of the bound product against the exact ones:
    # within the deviations of the stated worst case the library's decision
    # window is derived from (oz2_window.h; the window itself is twice as
    # wide on each side), and the measured hardware's narrower behaviour;
    # a split product adds its parts' sums, parts - 1 more roundings
    A, B = _bound_case(kind)
    r = run(A, B, 12, keep_ws=True)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True)
    check_stages(r, A, B, 12, st)
    assert _same(r.C, Chat)
    rA, rB = r.lines(8, np.uint32)
    kp = r.pads["kp"]
    parts = _bound_parts(A.shape[0], B.shape[1], kp)
    assert (parts > 1) == (kind == "split")
    Q = (kp + 7) // 8 + parts - 1
    # worst case (W): under by at most 7 2^-13 + Q 2^-23, over by at most
    # 7 2^-13 + 1.02 Q 2^-23
    down = 7 * 2.0 ** -13 + Q * 2.0 ** -23
    up = 7 * 2.0 ** -13 + 1.02 * Q * 2.0 ** -23
    # measured behaviour: truncation inside groups of 8, at most one upward
    # FP32 rounding per instruction of 64 k (and per addition of a part)
    hw_up = (kp / 64 + 2 + parts) * 2.0 ** -23
    worst_down = worst_up = 0.0
    for g32, exact18 in ((rA, st["r18"]), (rB, st["c18"])):
        g = g32.view(np.float32).astype(np.float64)
        exact = np.ldexp(exact18, -18)
        nz = exact > 0
        rel = g[nz] / exact[nz] - 1.0
        worst_down = max(worst_down, float(-rel.min()))
        worst_up = max(worst_up, float(rel.max()))
    print(f"bound {kind}: worst under {worst_down:.3e} (worst case {down:.3e}), worst over "
          f"{worst_up:.3e} (worst case {up:.3e}, measured model {hw_up:.3e}), paper's "
          f"(k-1) 2^-24 = {(kp - 1) * 2.0 ** -24:.3e}, exact fix-ups {r.fixups()}", flush=True)
    assert worst_down <= down and worst_up <= up
    assert worst_up <= hw_up


def test_deterministic_and_stream():
    A, B = _inputs(257, 255, 300, 1.0, 8000)
    r1 = run(A, B, 12)
    s = torch.cuda.Stream()
    r2 = run(A, B, 12, stream=s)
    assert _same(r1.C, r2.C)


def test_library_workspace_and_timing():
    # library-owned workspace (grown on demand), per-stage timing
    A, B = _inputs(300, 300, 300, 0.5, 9000)
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    oz.ozaki2_set_timing(True)
    C = oz.dgemm(tA, tB, 12)
    torch.cuda.synchronize()
    times = oz.ozaki2_get_stage_times()
    kt = oz.ozaki2_get_kernel_times()
    oz.ozaki2_set_timing(False)
    assert len(times) == 5 and all(t >= 0 for t in times) and times[1] > 0
    assert len(kt) == 6
    assert _same(C.cpu().numpy(), ref.emulate(A, B, 12))
    oz.ozaki2_release()


def test_workspace_too_small():
    A, B = _inputs(64, 64, 64, 1.0, 9100)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    oz.ozaki2_set_workspace(base, 512)
    try:
        tA = torch.from_numpy(A).cuda()
        tB = torch.from_numpy(B).cuda()
        tC = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
        st = oz.ozaki2_dgemm("N", "N", 64, 64, 64, 1.0, tA, 64, tB, 64, 0.0, tC, 64, 12)
    finally:
        oz.ozaki2_set_workspace(None, 0)
    assert st == 3


def test_full_size_sampled():
    # the benchmark workload: m = n = k = 8192, phi = 0.5, N = 12, in the
    # benchmark's launch configuration: every line's shift (the full oracle
    # scaling, from the whole bound product) and C on sampled rows (all
    # columns) and sampled columns (all rows)
    n = 8192
    s = config_seed(2, 0)
    print("full size: generating", flush=True)
    A = phi_matrix(n, n, 0.5, s)
    B = phi_matrix(n, n, 0.5, s + 1)
    print("full size: GPU", flush=True)
    r = run(A, B, 12, keep_ws="lines")
    assert r.status == 0
    rows = np.array([0, 1, 777, 4095, 8191])
    cols = np.arange(n)
    print("full size: oracle scaling", flush=True)
    sc = ref.scaling(A, B, 12)
    sA, sB = r.lines(0)
    assert np.array_equal(sA, sc["sA"]) and np.array_equal(sB, sc["sB"]), "shifts"
    print(f"full size: every shift equal; exact fix-ups {r.fixups()}", flush=True)
    print("full size: oracle rows", flush=True)
    Cs, _ = ref.products(sc, rows, cols)
    assert _same(r.C[rows], Cs)
    print("full size: oracle columns", flush=True)
    cols2 = np.array([5, 4096, 8190])
    Cs2, _ = ref.products(sc, np.arange(n), cols2)
    assert _same(r.C[:, cols2], Cs2)
    # FP64-level accuracy at the full-accuracy moduli count (phi = 0.5)
    hi, lo = dd_dot_rows(A[rows[:2]], B[:, :1024])
    err = normalised_error(r.C[rows[:2], :1024], hi, lo, np.abs(A[rows[:2]]), np.abs(B[:, :1024]))
    print(f"full size: normalised error {err:.3e}", flush=True)
    assert err <= 1e-15


def test_allocation_failure_is_reported():
    # OZ2_FAULT=alloc (read by the library once per process, so a child
    # process): every allocation the library would make fails; the calls
    # return OZ2_ERR_ALLOC and leave C untouched
    import os
    import subprocess
    import sys
    code = (
        "import torch, paper_2603_10634_amd as oz\n"
        "oz.ozaki2_set_stream(torch.cuda.current_stream())\n"
        "A = torch.ones((64, 64), dtype=torch.float64, device='cuda')\n"
        "C = torch.full((64, 64), 7.0, dtype=torch.float64, device='cuda')\n"
        "s1 = oz.ozaki2_dgemm('N', 'N', 64, 64, 64, 1.0, A, 64, A, 64, 0.0, C, 64, 12)\n"
        "s2 = oz.ozaki2_dgemm_batched(['N'], ['N'], [64], [64], [64], [1.0], [A], [64], [A],\n"
        "                             [64], [0.0], [C], [64], 12)\n"
        "torch.cuda.synchronize()\n"
        "print('STATUS', s1, s2, bool((C == 7.0).all()))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, OZ2_FAULT="alloc")
    print("allocation failure: child process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split("STATUS")[1].split() == ["2", "2", "True"]
    assert "allocat" in oz.ozaki2_status_string(2)
