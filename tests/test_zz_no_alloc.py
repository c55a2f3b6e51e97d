"""ozaki2_dgemm_noalloc (the entry point for callers that cannot allocate)
through the C ABI against ozaki2_dgemm on the same inputs: C bit for bit on
two calls in a row, the second smaller than the first (the fixed scratch
buffer keeps the first call's contents), with transposes and alpha/beta,
and with k split over several parts; a problem beyond the scratch buffer is
refused before anything is launched, and m/n blocking brings it back within
the buffer."""
import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from workloads import phi_matrix, to_colmajor

pytestmark = pytest.mark.gpu


def _call(entry, opA, opB, N, ta="N", tb="N", alpha=1.0, beta=0.0, Cin=None):
    m, k = opA.shape
    n = opB.shape[1]
    Ab, lda = to_colmajor(opA, ta, ld=(m if ta == "N" else k) + 3)
    Bb, ldb = to_colmajor(opB, tb, ld=(k if tb == "N" else n) + 1)
    Cm = np.zeros((m, n)) if Cin is None else Cin
    Cb, ldc = to_colmajor(Cm, "N", ld=m + 2, fill=7.0)
    dev = torch.device("cuda", 0)
    tA = torch.from_numpy(Ab).to(dev)
    tB = torch.from_numpy(Bb).to(dev)
    tC = torch.from_numpy(Cb).to(dev)
    oz.ozaki2_set_stream(torch.cuda.current_stream(dev))
    st = entry(ta, tb, m, n, k, alpha, tA, lda, tB, ldb, beta, tC, ldc, N)
    torch.cuda.synchronize(dev)
    return st, tC.cpu().numpy()


def _pair(opA, opB, N, **kw):
    st1, c1 = _call(oz.ozaki2_dgemm_noalloc, opA, opB, N, **kw)
    st2, c2 = _call(oz.ozaki2_dgemm, opA, opB, N, **kw)
    assert st1 == 0 and st2 == 0
    assert np.array_equal(c1.view(np.int64), c2.view(np.int64))


def test_noalloc_matches_dgemm_twice_smaller_second():
    A = phi_matrix(700, 900, 1.0, 71)
    B = phi_matrix(900, 520, 1.0, 72)
    print("noalloc: 700 x 520 x 900, N = 12", flush=True)
    _pair(A, B, 12)
    a = phi_matrix(300, 260, 2.0, 73)
    b = phi_matrix(260, 190, 2.0, 74)
    print("noalloc: 300 x 190 x 260, N = 14, T/T, alpha, beta", flush=True)
    Cin = phi_matrix(300, 190, 0.5, 75)
    _pair(a, b, 14, ta="T", tb="T", alpha=-1.5, beta=0.25, Cin=Cin)


def test_noalloc_fast_mode_and_int8():
    A = phi_matrix(257, 333, 1.0, 81)
    B = phi_matrix(333, 129, 1.0, 82)
    try:
        assert oz.ozaki2_set_mode("fast") == 0
        print("noalloc: fast mode N = 13", flush=True)
        _pair(A, B, 13)
        assert oz.ozaki2_set_mode("accurate") == 0
        assert oz.ozaki2_set_moduli_list("int8") == 0
        print("noalloc: int8 N = 15", flush=True)
        _pair(A, B, 15, ta="T")
    finally:
        oz.ozaki2_set_mode("accurate")
        oz.ozaki2_set_moduli_list("hybrid")


def test_noalloc_split_products_and_bound():
    # one output tile with a long k: the products run in k parts (plane
    # copies) and the bound product in parts summed by a second launch, all
    # inside the scratch buffer; then a smaller call on the same buffer
    m, n, k = 256, 256, 8192
    parts, bparts = oz.ozaki2_workspace_parts(m, n, k, 12)
    assert parts > 1 and bparts > 1
    assert oz.ozaki2_workspace_bytes(m, n, k, 12) <= oz.NOALLOC_SCRATCH_BYTES
    A = phi_matrix(m, k, 1.0, 95)
    B = phi_matrix(k, n, 1.0, 96)
    print(f"noalloc: {m} x {n} x {k}, {parts} product parts, {bparts} bound parts", flush=True)
    _pair(A, B, 12)
    a = phi_matrix(100, 5000, 1.0, 97)
    b = phi_matrix(5000, 90, 1.0, 98)
    print("noalloc: 100 x 90 x 5000", flush=True)
    _pair(a, b, 12, ta="T")


def test_noalloc_refuses_beyond_scratch_and_blocking_fits():
    m = n = 2816
    k = 2048
    assert oz.ozaki2_workspace_bytes(m, n, k, 12) > oz.NOALLOC_SCRATCH_BYTES
    A = phi_matrix(m, k, 0.5, 91)
    B = phi_matrix(k, n, 0.5, 92)
    print("noalloc: too large for the scratch buffer", flush=True)
    st, c = _call(oz.ozaki2_dgemm_noalloc, A, B, 12)
    assert st == 6                                    # OZ2_ERR_SCRATCH
    cv = c.reshape(n, m + 2)                           # C untouched: zeros, padding 7
    assert np.all(cv[:, :m] == 0.0) and np.all(cv[:, m:] == 7.0)
    try:
        assert oz.ozaki2_set_blocking(1024, 1024) == 0
        assert oz.ozaki2_workspace_bytes(m, n, k, 12) <= oz.NOALLOC_SCRATCH_BYTES
        print("noalloc: 1024 x 1024 blocks", flush=True)
        st1, c1 = _call(oz.ozaki2_dgemm_noalloc, A, B, 12)
    finally:
        oz.ozaki2_set_blocking(0, 0)
    st2, c2 = _call(oz.ozaki2_dgemm, A, B, 12)
    assert st1 == 0 and st2 == 0
    assert np.array_equal(c1.view(np.int64), c2.view(np.int64))
