"""Fast mode (Section III-E: scale exponents from the Cauchy-Schwarz bound)
on the GPU against the oracle's fast mode, through the C ABI: every stored
intermediate and C bit for bit on ragged shapes, all storage orders, alpha /
beta, zero and non-finite lines, the largest k, batched and graph calls, and
the full-size workload on sampled outputs."""
import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import phi_matrix, normal_matrix, config_seed, batch_shapes, to_colmajor
from workloads.reference import dd_dot_rows, normalised_error

from gpu_util import run, check_stages, check_sampled, sample_lines

pytestmark = pytest.mark.gpu


def _inputs(m, n, k, phi, seed):
    if phi is None:
        return normal_matrix(m, k, seed), normal_matrix(k, n, seed + 1)
    return phi_matrix(m, k, phi, seed), phi_matrix(k, n, phi, seed + 1)


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


def test_mode_setting():
    assert oz.ozaki2_get_mode() == oz.MODE_ACCURATE
    assert oz.ozaki2_set_mode("fast") == 0 and oz.ozaki2_get_mode() == oz.MODE_FAST
    assert oz.ozaki2_set_mode(7) == -1 and oz.ozaki2_get_mode() == oz.MODE_FAST
    assert oz.ozaki2_set_mode("accurate") == 0 and oz.ozaki2_get_mode() == oz.MODE_ACCURATE


@pytest.mark.parametrize("N", [1, 2, 6, 7, 12, 13, 20, 33])
def test_fast_stage_parity_ragged(N):
    print(f"fast stage parity N={N} shape=(300, 200, 700)", flush=True)
    A, B = _inputs(300, 200, 700, 1.0, 1100 + N)
    r = run(A, B, N, keep_ws=True, mode="fast")
    assert r.status == 0
    Chat, st = ref.emulate(A, B, N, keep_stages=True, mode="fast")
    check_stages(r, A, B, N, st, mode="fast")
    assert _same(r.C, Chat)


@pytest.mark.parametrize("phi", [None, 0.5, 4.0, 6.0])
@pytest.mark.parametrize("shape", [(256, 256, 256), (129, 385, 200), (64, 64, 1),
                                   (1, 300, 513), (520, 1, 77)])
def test_fast_parity_shapes(phi, shape):
    m, n, k = shape
    print(f"fast parity shape={shape} phi={phi}", flush=True)
    A, B = _inputs(m, n, k, phi, 2100 + m + n + k)
    r = run(A, B, 13, keep_ws=True, mode="fast")
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 13, keep_stages=True, mode="fast")
    check_stages(r, A, B, 13, st, mode="fast")
    assert _same(r.C, Chat)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
def test_fast_transposes_alpha_beta(ta, tb):
    print(f"fast transposes {ta}{tb}", flush=True)
    A, B = _inputs(190, 260, 333, 2.0, 3100)
    Cin = phi_matrix(190, 260, 1.0, 3102)
    want = ref.combine_alpha_beta(ref.emulate(A, B, 13, mode="fast"), -1.25, 0.5, Cin)
    r = run(A, B, 13, transA=ta, transB=tb, alpha=-1.25, beta=0.5, Cin=Cin, pad=(3, 5, 2),
            mode="fast")
    assert r.status == 0
    assert _same(r.C, want)
    Cb = r.Cbuf.reshape(-1, r.ldc)
    assert np.all(Cb[:, r.m:] == 7.0)


def test_fast_zero_nonfinite_subnormal():
    A, B = _inputs(150, 140, 90, 1.0, 5300)
    A[3, :] = 0.0
    B[:, 7] = 0.0
    A[10, 5] = np.inf
    B[20, 9] = np.nan
    A[0] *= 2.0 ** -1060
    A[2] *= 2.0 ** 900
    B[:, 1] *= 2.0 ** -1000
    r = run(A, B, 12, keep_ws=True, mode="fast")
    assert r.status == 0
    Chat, st = ref.emulate(A, B, 12, keep_stages=True, mode="fast")
    check_stages(r, A, B, 12, st, mode="fast")
    assert _same(r.C, Chat)
    assert np.all(np.isnan(r.C[10])) and np.all(np.isnan(r.C[:, 9]))


def test_fast_largest_norms_exact():
    # k = 2^18 (the largest k) with every scaled entry rounding up to 256: the
    # squared norms reach 2^18 x 2^34 = 2^52, the top of the exact range.
    # Random low mantissa bits make C depend on the exact shifts.
    k = 1 << 18
    print(f"fast largest norms k={k}", flush=True)
    rng = np.random.default_rng(5400)
    A = 255.5 / 128.0 + rng.uniform(0.0, 2.0 ** -12, (8, k))
    B = 255.5 / 128.0 + rng.uniform(0.0, 2.0 ** -12, (k, 8))
    A[1::2, ::3] *= -1.0
    A[5] *= 2.0 ** -40
    B[:, 3] = np.ldexp(phi_matrix(k, 1, 1.0, 5401)[:, 0], 3)
    r = run(A, B, 13, keep_ws="lines", mode="fast")
    assert r.status == 0
    sc = ref.scaling(A, B, 13, mode="fast")
    assert int(sc["r18"][0]) == 2 ** 52 and int(sc["c18"][0]) == 2 ** 52
    eA, eB = r.lines(2)
    assert np.array_equal(eA, sc["e"]) and np.array_equal(eB, sc["f"])
    Chat, _ = ref.products(sc, np.arange(8), np.arange(8))
    assert _same(r.C, Chat)


def test_fast_equals_accurate_when_tight():
    # random signs times one power of two per line: Abar = Bbar = 128, so the
    # Cauchy-Schwarz bound is attained and both modes give the same C
    rng = np.random.default_rng(5500)
    m, k, n = 300, 513, 260
    A = rng.choice([-1.0, 1.0], (m, k)) * np.ldexp(1.0, rng.integers(-30, 30, (m, 1)))
    B = rng.choice([-1.0, 1.0], (k, n)) * np.ldexp(1.0, rng.integers(-30, 30, (1, n)))
    rf = run(A, B, 12, keep_ws=True, mode="fast")
    ra = run(A, B, 12, keep_ws=True)
    assert rf.status == 0 and ra.status == 0
    assert np.array_equal(rf.lines(2)[0], ra.lines(2)[0])
    assert _same(rf.C, ra.C)
    assert _same(rf.C, ref.emulate(A, B, 12, mode="fast"))


def _batched(As, Bs, N, mode):
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
    assert oz.ozaki2_set_mode(mode) == 0
    try:
        st = oz.ozaki2_dgemm_batched(["N"] * cnt, ["N"] * cnt, m, n, k, [1.0] * cnt, tA,
                                     [max(1, x) for x in m], tB, [max(1, x) for x in k],
                                     [0.0] * cnt, tC, [max(1, x) for x in m], N)
        torch.cuda.synchronize()
    finally:
        oz.ozaki2_set_mode("accurate")
    assert st == 0
    return [c.cpu().numpy().reshape(nn, mm).T for c, mm, nn in zip(tC, m, n)]


def test_fast_batched_and_mode_switch():
    shapes = batch_shapes(12, 32, 600, seed=5600)
    As = [phi_matrix(m, k, 2.0, 5601 + q) for q, (m, n, k) in enumerate(shapes)]
    Bs = [phi_matrix(k, n, 2.0, 5701 + q) for q, (m, n, k) in enumerate(shapes)]
    print(f"fast batched shapes={shapes}", flush=True)
    Cf = _batched(As, Bs, 13, "fast")
    Ca = _batched(As, Bs, 13, "accurate")   # same arguments, other mode: its own plan
    Cf2 = _batched(As, Bs, 13, "fast")
    for q in range(len(As)):
        assert _same(Cf[q], ref.emulate(As[q], Bs[q], 13, mode="fast")), q
        assert _same(Ca[q], ref.emulate(As[q], Bs[q], 13)), q
        assert _same(Cf2[q], Cf[q]), q


def test_fast_graph_replays():
    A, B = _inputs(300, 280, 400, 1.0, 5800)
    dev = torch.device("cuda", 0)
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    want_f = ref.emulate(A, B, 13, mode="fast")
    want_a = ref.emulate(A, B, 13)
    oz.ozaki2_set_graph(True)
    try:
        C = torch.empty((300, 280), dtype=torch.float64, device=dev)
        for rep in range(3):
            oz.dgemm(tA, tB, 13, C=C, mode="fast")
            torch.cuda.synchronize()
            assert _same(C.cpu().numpy(), want_f), rep
            oz.dgemm(tA, tB, 13, C=C, mode="accurate")
            torch.cuda.synchronize()
            assert _same(C.cpu().numpy(), want_a), rep
    finally:
        oz.ozaki2_set_graph(False)


def test_fast_full_size_sampled():
    # m = n = k = 8192, phi = 0.5, 13 moduli (fast): shifts of sampled lines,
    # sampled outputs bit for bit, normalised error against double-double
    n = 8192
    s = config_seed(2, 0)
    print("fast full size: generating", flush=True)
    A = phi_matrix(n, n, 0.5, s)
    B = phi_matrix(n, n, 0.5, s + 1)
    rows = sample_lines(n, 20, 11)
    cols = sample_lines(n, 20, 12)
    check_sampled(A, B, 13, rows, cols, mode="fast", label="fast full size")
