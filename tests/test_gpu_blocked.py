"""m/n-blocked calls (ozaki2_set_blocking; Section IV-C's workspace blocking)
through the C ABI: the scale exponents come from the whole problem, so a
blocked call must equal the unblocked call and the oracle bit for bit, for
ragged block grids, every storage order, alpha/beta, both modes, all three
modulus lists, special lines, graph replays and the 8192^3 workload."""
import time

import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import phi_matrix, normal_matrix, config_seed

from gpu_util import run

pytestmark = pytest.mark.gpu


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


@pytest.mark.parametrize("blocking", [(256, 256), (512, 256), (256, 0), (0, 512)])
def test_blocked_equals_unblocked_and_oracle(blocking):
    print(f"blocked {blocking} shape=(700, 600, 300)", flush=True)
    A = phi_matrix(700, 300, 1.0, 7100)
    B = phi_matrix(300, 600, 1.0, 7101)
    rb = run(A, B, 12, blocking=blocking)
    ru = run(A, B, 12)
    assert rb.status == 0 and ru.status == 0
    assert _same(rb.C, ru.C)
    assert _same(rb.C, ref.emulate(A, B, 12))


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
def test_blocked_transposes_alpha_beta(ta, tb):
    A = phi_matrix(530, 290, 2.0, 7200)
    B = phi_matrix(290, 777, 2.0, 7201)
    Cin = phi_matrix(530, 777, 1.0, 7202)
    want = ref.combine_alpha_beta(ref.emulate(A, B, 12), 1.5, -0.25, Cin)
    r = run(A, B, 12, transA=ta, transB=tb, alpha=1.5, beta=-0.25, Cin=Cin, pad=(1, 2, 3),
            blocking=(256, 512))
    assert r.status == 0
    assert _same(r.C, want)
    Cb = r.Cbuf.reshape(-1, r.ldc)
    assert np.all(Cb[:, r.m:] == 7.0)


@pytest.mark.parametrize("mode,moduli,N", [("fast", "hybrid", 13), ("accurate", "karatsuba", 13),
                                           ("accurate", "int8", 14), ("fast", "int8", 16)])
def test_blocked_modes_and_lists(mode, moduli, N):
    A = normal_matrix(600, 400, 7300)
    B = normal_matrix(400, 520, 7301)
    A[5, :] = 0.0
    A[300, 7] = np.inf
    B[:, 260] = 0.0
    B[11, 511] = np.nan
    r = run(A, B, N, mode=mode, moduli=moduli, blocking=(256, 256))
    assert r.status == 0
    assert _same(r.C, ref.emulate(A, B, N, mode=mode, moduli_set=moduli))


def test_blocked_graph_replays():
    A = phi_matrix(640, 300, 1.0, 7400)
    B = phi_matrix(300, 700, 1.0, 7401)
    want = ref.emulate(A, B, 12)
    dev = torch.device("cuda", 0)
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    C = torch.empty((640, 700), dtype=torch.float64, device=dev)
    assert oz.ozaki2_set_blocking(256, 256) == 0
    oz.ozaki2_set_graph(True)
    try:
        for rep in range(3):
            C.fill_(3.0)
            oz.dgemm(tA, tB, 12, C=C)
            torch.cuda.synchronize()
            assert _same(C.cpu().numpy(), want), rep
    finally:
        oz.ozaki2_set_graph(False)
        oz.ozaki2_set_blocking(0, 0)


def test_blocked_full_size_equals_unblocked():
    # 8192^3, N = 12, 4096 x 4096 blocks against the unblocked call, bit for
    # bit, with the time of each (library-owned workspace)
    n = 8192
    s = config_seed(2, 0)
    print("blocked full size: generating", flush=True)
    dev = torch.device("cuda", 0)
    tA = torch.from_numpy(phi_matrix(n, n, 0.5, s)).to(dev)
    tB = torch.from_numpy(phi_matrix(n, n, 0.5, s + 1)).to(dev)
    out = {}
    for blk in (0, 4096):
        assert oz.ozaki2_set_blocking(blk, blk) == 0
        try:
            C = oz.dgemm(tA, tB, 12)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                C = oz.dgemm(tA, tB, 12)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 3
            out[blk] = C.cpu().numpy()
            print(f"blocked full size: blocks {blk}: {dt * 1e3:.2f} ms, workspace "
                  f"{oz.ozaki2_workspace_bytes(n, n, n, 12) / 1e9:.2f} GB", flush=True)
        finally:
            oz.ozaki2_set_blocking(0, 0)
            oz.ozaki2_release()
    assert _same(out[0], out[4096])
