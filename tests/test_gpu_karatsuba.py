"""The Karatsuba-only modulus list (Section III-B: 513, 512, 511, 509, 505,
..., every modulus with the Karatsuba split) on the GPU against the oracle
with the same list, through the C ABI.  513 = 3^3 19 and 505 = 5 101 run their
three products in the other pass order (15 is not invertible modulo them),
512 is even; all three are among the first five moduli."""
import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import phi_matrix, normal_matrix, config_seed, batch_shapes, to_colmajor
from workloads.reference import dd_dot_rows, normalised_error

from gpu_util import run, check_stages, check_sampled, sample_lines, split

pytestmark = pytest.mark.gpu

KA = "karatsuba"


def _inputs(m, n, k, phi, seed):
    if phi is None:
        return normal_matrix(m, k, seed), normal_matrix(k, n, seed + 1)
    return phi_matrix(m, k, phi, seed), phi_matrix(k, n, phi, seed + 1)


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


@pytest.mark.parametrize("N", [1, 2, 3, 5, 12, 13, 20, 33])
def test_karatsuba_stage_parity_ragged(N):
    print(f"karatsuba-only stage parity N={N} shape=(300, 200, 700)", flush=True)
    A, B = _inputs(300, 200, 700, 1.0, 1200 + N)
    r = run(A, B, N, keep_ws=True, moduli=KA)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, N, keep_stages=True, moduli_set=KA)
    check_stages(r, A, B, N, st, moduli=KA)
    assert _same(r.C, Chat)


@pytest.mark.parametrize("phi", [None, 4.0])
@pytest.mark.parametrize("shape", [(129, 385, 200), (64, 64, 1), (1, 300, 513)])
def test_karatsuba_shapes_fast_mode(phi, shape):
    m, n, k = shape
    print(f"karatsuba-only fast shape={shape} phi={phi}", flush=True)
    A, B = _inputs(m, n, k, phi, 2200 + m + n + k)
    r = run(A, B, 13, keep_ws=True, mode="fast", moduli=KA)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 13, keep_stages=True, mode="fast", moduli_set=KA)
    check_stages(r, A, B, 13, st, mode="fast", moduli=KA)
    assert _same(r.C, Chat)


@pytest.mark.parametrize("ta,tb", [("N", "T"), ("T", "N")])
def test_karatsuba_transposes_alpha_beta(ta, tb):
    A, B = _inputs(190, 260, 333, 1.0, 3200)
    Cin = phi_matrix(190, 260, 1.0, 3202)
    want = ref.combine_alpha_beta(ref.emulate(A, B, 13, moduli_set=KA), 0.75, -2.0, Cin)
    r = run(A, B, 13, transA=ta, transB=tb, alpha=0.75, beta=-2.0, Cin=Cin, pad=(2, 3, 1),
            moduli=KA)
    assert r.status == 0
    assert _same(r.C, want)


def _constant_case(k, N):
    """Constant op(A) = c/128 and op(B) = d/128 (c, d in [128, 256)) chosen so
    that a digit product of 16 x 16 occurs for one of the moduli 513, 512,
    505: that product's FP32 sum then reaches 256 k = 2^23 at k = 2^15, added
    to a folded accumulator of magnitude up to 256."""
    for c in range(128, 256):
        for d in (c, 255, 200, 129):
            A = np.full((1, k), c / 128.0)
            B = np.full((k, 1), d / 128.0)
            _, st = ref.emulate(A, B, N, keep_stages=True, moduli_set=KA)
            for pm in st["per_modulus"]:
                if pm["p"] not in (513, 512, 505):
                    continue
                for x in range(3):
                    if abs(int(pm["dA"][x][0, 0]) * int(pm["dB"][x][0, 0])) == 256:
                        return c / 128.0, d / 128.0
    raise AssertionError("no extreme-digit constant found")


def test_karatsuba_extreme_digit_sums_exact():
    k = 32768
    a, b = _constant_case(k, 5)
    print(f"karatsuba-only extreme digits a={a} b={b}", flush=True)
    A = np.full((64, k), a)
    B = np.full((k, 96), b)
    A[1::2] *= -1.0
    with split(1):   # one k part: a single accumulation over all 2^15
        r = run(A, B, 5, keep_ws=True, moduli=KA)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 5, keep_stages=True, moduli_set=KA)
    check_stages(r, A, B, 5, st, moduli=KA)
    assert _same(r.C, Chat)


def test_karatsuba_long_k():
    k = 65536 + 300
    A, B = _inputs(40, 72, k, 1.0, 6100)
    r = run(A, B, 13, keep_ws=True, moduli=KA)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 13, keep_stages=True, moduli_set=KA)
    P = r.planes(13, [pm["p"] for pm in st["per_modulus"]])
    for l, plane in enumerate(st["planes"]):
        assert np.array_equal(P[l, :72, :40].T.astype(np.int64), plane), f"plane {l}"
    assert _same(r.C, Chat)


def _batched(As, Bs, N, moduli):
    dev = torch.device("cuda", 0)
    tA = [torch.from_numpy(to_colmajor(a, "N")[0].copy()).to(dev) for a in As]
    tB = [torch.from_numpy(to_colmajor(b, "N")[0].copy()).to(dev) for b in Bs]
    tC = [torch.zeros(a.shape[0] * b.shape[1], dtype=torch.float64, device=dev)
          for a, b in zip(As, Bs)]
    cnt = len(As)
    m = [a.shape[0] for a in As]
    k = [a.shape[1] for a in As]
    n = [b.shape[1] for b in Bs]
    oz.ozaki2_set_stream(torch.cuda.current_stream(dev))
    assert oz.ozaki2_set_moduli_list(moduli) == 0
    try:
        st = oz.ozaki2_dgemm_batched(["N"] * cnt, ["N"] * cnt, m, n, k, [1.0] * cnt, tA,
                                     [max(1, x) for x in m], tB, [max(1, x) for x in k],
                                     [0.0] * cnt, tC, [max(1, x) for x in m], N)
        torch.cuda.synchronize()
    finally:
        oz.ozaki2_set_moduli_list("hybrid")
    assert st == 0
    return [c.cpu().numpy().reshape(nn, mm).T for c, mm, nn in zip(tC, m, n)]


def test_karatsuba_batched_list_switch():
    shapes = batch_shapes(10, 32, 500, seed=6200)
    As = [phi_matrix(m, k, 1.0, 6201 + q) for q, (m, n, k) in enumerate(shapes)]
    Bs = [phi_matrix(k, n, 1.0, 6301 + q) for q, (m, n, k) in enumerate(shapes)]
    print(f"karatsuba-only batched shapes={shapes}", flush=True)
    Ck = _batched(As, Bs, 13, KA)
    Ch = _batched(As, Bs, 13, "hybrid")   # same arguments, other list: its own plan
    for q in range(len(As)):
        assert _same(Ck[q], ref.emulate(As[q], Bs[q], 13, moduli_set=KA)), q
        assert _same(Ch[q], ref.emulate(As[q], Bs[q], 13)), q


def test_karatsuba_full_size_sampled():
    # m = n = k = 8192, phi = 0.5, 13 moduli (karatsuba-only): shifts of sampled lines,
    # sampled outputs bit for bit, normalised error against double-double
    n = 8192
    s = config_seed(2, 0)
    print("karatsuba-only full size: generating", flush=True)
    A = phi_matrix(n, n, 0.5, s)
    B = phi_matrix(n, n, 0.5, s + 1)
    rows = sample_lines(n, 20, 11)
    cols = sample_lines(n, 20, 12)
    check_sampled(A, B, 13, rows, cols, moduli=KA, label="karatsuba-only full size")
