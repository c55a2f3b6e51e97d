"""The INT8 arm (Section II: moduli 256, 255, 253, 251, 247, ..., one INT8
operand and one INT8 product per modulus, INT32 accumulation) on the GPU
against the oracle's INT8 arm, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import phi_matrix, normal_matrix, config_seed, batch_shapes, to_colmajor
from workloads.reference import dd_dot_rows, normalised_error

from gpu_util import run, check_stages, check_sampled, sample_lines, split

pytestmark = pytest.mark.gpu

I8 = "int8"


def _inputs(m, n, k, phi, seed):
    if phi is None:
        return normal_matrix(m, k, seed), normal_matrix(k, n, seed + 1)
    return phi_matrix(m, k, phi, seed), phi_matrix(k, n, phi, seed + 1)


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


@pytest.mark.parametrize("N", [1, 2, 5, 14, 15, 16, 20, 33])
def test_int8_stage_parity_ragged(N):
    print(f"int8 stage parity N={N} shape=(300, 200, 700)", flush=True)
    A, B = _inputs(300, 200, 700, 1.0, 1300 + N)
    r = run(A, B, N, keep_ws=True, moduli=I8)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, N, keep_stages=True, moduli_set=I8)
    check_stages(r, A, B, N, st, moduli=I8)
    assert _same(r.C, Chat)


@pytest.mark.parametrize("phi", [None, 4.0])
@pytest.mark.parametrize("shape", [(129, 385, 200), (64, 64, 1), (1, 300, 513)])
def test_int8_shapes_fast_mode(phi, shape):
    m, n, k = shape
    print(f"int8 fast shape={shape} phi={phi}", flush=True)
    A, B = _inputs(m, n, k, phi, 2300 + m + n + k)
    r = run(A, B, 15, keep_ws=True, mode="fast", moduli=I8)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 15, keep_stages=True, mode="fast", moduli_set=I8)
    check_stages(r, A, B, 15, st, mode="fast", moduli=I8)
    assert _same(r.C, Chat)


@pytest.mark.parametrize("ta,tb", [("N", "T"), ("T", "N")])
def test_int8_transposes_alpha_beta(ta, tb):
    A, B = _inputs(190, 260, 333, 1.0, 3300)
    Cin = phi_matrix(190, 260, 1.0, 3302)
    want = ref.combine_alpha_beta(ref.emulate(A, B, 14, moduli_set=I8), 0.75, -2.0, Cin)
    r = run(A, B, 14, transA=ta, transB=tb, alpha=0.75, beta=-2.0, Cin=Cin, pad=(2, 3, 1),
            moduli=I8)
    assert r.status == 0
    assert _same(r.C, want)


def _constant_case(k):
    """A constant x = 1 + 2^-t whose integer a' = 2^s + 2^(s - t) has the
    residue -128 modulo 256 (t = s - 7, s the shift the scaling picks at this
    k): every INT8 product of that modulus is (-128)^2 = 2^14, so a chunk of
    k = 2^15 sums to 2^29 in INT32."""
    for t in range(9, 52):
        x = 1.0 + 2.0 ** -t
        A = np.full((1, k), x)
        _, st = ref.emulate(A, A.T.copy(), 14, keep_stages=True, moduli_set=I8)
        pm = st["per_modulus"][0]
        if pm["p"] == 256 and int(pm["uA"][0, 0]) == -128 and int(pm["uB"][0, 0]) == -128:
            return x
    raise AssertionError("no extreme-residue constant found")


@pytest.mark.parametrize("k", [32768, 65536 + 256])
def test_int8_extreme_sums_exact(k):
    a = _constant_case(k)
    print(f"int8 extreme residues a={a} k={k}", flush=True)
    A = np.full((64, k), a)
    B = np.full((k, 96), a)
    A[1::2] *= -1.0
    with split(1):   # the fewest k parts: accumulations of up to 2^15
        r = run(A, B, 14, keep_ws=True, moduli=I8)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 14, keep_stages=True, moduli_set=I8)
    assert int(st["per_modulus"][0]["uA"][0, 0]) == -128
    assert abs(int(st["per_modulus"][0]["uA"][1, 0])) == 128
    check_stages(r, A, B, 14, st, moduli=I8)
    assert _same(r.C, Chat)


def test_int8_long_k():
    k = 65536 + 300
    A, B = _inputs(40, 72, k, 1.0, 6400)
    r = run(A, B, 15, keep_ws=True, moduli=I8)
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 15, keep_stages=True, moduli_set=I8)
    P = r.planes(15, [pm["p"] for pm in st["per_modulus"]])
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


def test_int8_batched_list_switch():
    shapes = batch_shapes(10, 32, 500, seed=6500)
    As = [phi_matrix(m, k, 1.0, 6501 + q) for q, (m, n, k) in enumerate(shapes)]
    Bs = [phi_matrix(k, n, 1.0, 6601 + q) for q, (m, n, k) in enumerate(shapes)]
    print(f"int8 batched shapes={shapes}", flush=True)
    Ck = _batched(As, Bs, 14, I8)
    Ch = _batched(As, Bs, 14, "hybrid")   # same arguments, other list: its own plan
    for q in range(len(As)):
        assert _same(Ck[q], ref.emulate(As[q], Bs[q], 14, moduli_set=I8)), q
        assert _same(Ch[q], ref.emulate(As[q], Bs[q], 14)), q


def test_int8_full_size_sampled():
    # m = n = k = 8192, phi = 0.5, 14 moduli (int8): shifts of sampled lines,
    # sampled outputs bit for bit, normalised error against double-double
    n = 8192
    s = config_seed(2, 0)
    print("int8 full size: generating", flush=True)
    A = phi_matrix(n, n, 0.5, s)
    B = phi_matrix(n, n, 0.5, s + 1)
    rows = sample_lines(n, 20, 11)
    cols = sample_lines(n, 20, 12)
    check_sampled(A, B, 14, rows, cols, moduli=I8, label="int8 full size")
