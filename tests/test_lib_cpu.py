"""Host-side checks of liboz2.so that need no GPU: the library loads, exports
every function include/ozaki2.h declares, uses the same moduli as the oracle,
lays its workspace out consistently and rejects invalid arguments before it
touches a device."""
import ctypes
import subprocess

import pytest

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref


@pytest.fixture(scope="module")
def L():
    return oz.lib()


def test_every_header_function_is_exported(L):
    names = oz.header_functions()
    assert "ozaki2_dgemm" in names and len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", oz.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_moduli_match_oracle(L):
    for N in range(1, 34):
        p, kinds = oz.ozaki2_moduli(N)
        want = ref.hybrid_moduli(N)
        assert p == [q for q, _, _ in want]
        assert kinds == [0 if k == "square" else 1 for _, k, _ in want]
    with pytest.raises(ValueError):
        oz.ozaki2_moduli(0)
    with pytest.raises(ValueError):
        oz.ozaki2_moduli(34)


@pytest.mark.parametrize("shape", [(1, 1, 1), (300, 200, 700), (8192, 8192, 8192),
                                   (1024, 1024, 65536), (16384, 16384, 1024)])
@pytest.mark.parametrize("N", [1, 6, 7, 12, 20, 33])
def test_workspace_layout(shape, N):
    m, n, k = shape
    off, pads = oz.ozaki2_workspace_layout(m, n, k, N)
    mp, np_, kp, M = pads["mp"], pads["np"], pads["kp"], pads["M"]
    assert mp % 256 == 0 and np_ % 256 == 0 and kp % 256 == 0
    assert mp >= m and np_ >= n and kp >= k and mp - m < 256 and kp - k < 256
    assert M == sum(2 if kd == "square" else 3 for _, kd, _ in ref.hybrid_moduli(N))
    total = oz.ozaki2_workspace_bytes(m, n, k, N)
    assert all(o % 256 == 0 for o in off)
    sizes = {0: 4 * (mp + np_), 1: 4 * (mp + np_), 2: 4 * (mp + np_), 3: mp * kp,
             4: np_ * kp, 5: M * mp * kp, 6: M * np_ * kp, 7: 2 * N * mp * np_,
             8: 4 * (mp + np_), 9: 4 * (mp + np_)}
    assert len(off) == 11 and off[10] % 256 == 0
    spans = sorted((off[i], off[i] + sizes[i]) for i in range(8))
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0                      # no overlap
    assert max(e for _, e in spans) <= total


def _min_parts(k):
    """Every k part is at most 2^15 long (one exact FP32 accumulation)."""
    return -(-((max(k, 1) + 255) // 256 * 256) // 2 ** 15)


def _rule_parts(m, n, k, N):
    """k parts of a single call's residue products: from the minimum up to 8
    parts (at least 2048 k each beyond the minimum), the fewest that
    minimise sum over modulus kinds of
    ceil(tiles * moduli of the kind * parts / 256) / parts."""
    pad = lambda x: (max(x, 1) + 255) // 256 * 256
    tiles = pad(m) // 256 * (pad(n) // 256)
    kinds = [sum(1 for _, kd, _ in ref.hybrid_moduli(N) if kd == want)
             for want in ("square", "karatsuba")]
    lo = _min_parts(k)
    best, best_cost = lo, None
    for parts in range(lo, 9):
        if parts > lo and pad(k) // parts < 2048:
            break
        cost = sum(-(-tiles * c * parts // 256) / parts for c in kinds if c)
        if best_cost is None or cost < best_cost:
            best, best_cost = parts, cost
    return best


def _bound_parts(m, n, k):
    """k parts of a single call's bound product: with fewer than 128 output
    tiles and k of at least 8192, up to 16 parts of at least 4096 k, about
    one workgroup per CU (256)."""
    pad = lambda x: (max(x, 1) + 255) // 256 * 256
    tiles = pad(m) // 256 * (pad(n) // 256)
    if tiles >= 128 or pad(k) < 8192:
        return 1
    return min(-(-256 // tiles), pad(k) // 4096, 16)


@pytest.mark.parametrize("shape,N,want", [
    ((8192, 8192, 8192), 12, 1), ((16384, 16384, 1024), 12, 1), ((4096, 4096, 4096), 12, 1),
    ((1024, 1024, 65536), 12, 8), ((40, 72, 65536), 12, 8), ((300, 200, 4096), 12, 2),
    ((300, 200, 2048), 12, 1), ((2048, 2048, 16384), 12, 2), ((1024, 1024, 65536), 7, 8),
    ((8192, 8192, 65536), 12, 2), ((4096, 4096, 2 ** 18), 12, 8), ((4096, 4096, 40000), 12, 2),
    ((1024, 1024, 65536), 1, 8), ((256, 256, 2 ** 18), 1, 8)])
def test_single_call_split(shape, N, want):
    m, n, k = shape
    pad = lambda x: (x + 255) // 256 * 256
    assert _rule_parts(m, n, k, N) == want
    off, pads = oz.ozaki2_workspace_layout(m, n, k, N)
    plane = 2 * N * pads["mp"] * pads["np"]
    # the last region holds the plane copies, or the split bound product's
    # part sums when those are larger (they are done before the planes)
    bound = 4 * pads["mp"] * pads["np"] * _bound_parts(m, n, k)
    size = lambda parts: off[7] + pad(max(plane * parts, bound))
    assert oz.ozaki2_workspace_bytes(m, n, k, N) == size(want)
    try:
        for forced in (1, 3, 8):
            assert oz.ozaki2_set_split(forced) == 0
            got = max(_min_parts(k), min(forced, pads["kp"] // 256))
            assert oz.ozaki2_workspace_bytes(m, n, k, N) == size(got)
        # refused values leave the setting (8) unchanged
        assert oz.ozaki2_set_split(9) == -1 and oz.ozaki2_set_split(-1) == -1
        assert oz.ozaki2_workspace_bytes(m, n, k, N) == size(min(8, pads["kp"] // 256))
    finally:
        oz.ozaki2_set_split(0)
    assert oz.ozaki2_workspace_bytes(m, n, k, N) == size(want)


@pytest.mark.parametrize("entry", ["ozaki2_dgemm", "ozaki2_dgemm_noalloc"])
def test_argument_errors(L, entry):
    d = 0  # no pointer is dereferenced on these paths
    call = getattr(oz, entry)
    assert call("X", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 12) == -1
    assert call("N", "Q", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 12) == -2
    assert call("N", "N", -1, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 12) == -3
    assert call("N", "N", 4, -1, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 12) == -4
    assert call("N", "N", 4, 4, -1, 1.0, d, 4, d, 4, 0.0, d, 4, 12) == -5
    assert call("N", "N", 4, 4, 4, 1.0, d, 3, d, 4, 0.0, d, 4, 12) == -8
    assert call("T", "N", 4, 4, 5, 1.0, d, 4, d, 5, 0.0, d, 4, 12) == -8
    assert call("N", "N", 4, 4, 4, 1.0, d, 4, d, 3, 0.0, d, 4, 12) == -10
    assert call("N", "T", 4, 5, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 12) == -10
    assert call("N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 3, 12) == -13
    assert call("N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 0) == -14
    assert call("N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, 34) == -14
    # empty output: nothing to do, success without a device
    assert call("N", "N", 0, 4, 4, 1.0, d, 1, d, 4, 0.0, d, 1, 12) == 0
    assert call("n", "t", 4, 0, 4, 1.0, d, 4, d, 1, 0.0, d, 4, 12) == 0


def test_no_device_reported_on_cpu(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert oz.ozaki2_dgemm("N", "N", 4, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4, 12) == 5
    assert oz.ozaki2_dgemm_noalloc("N", "N", 4, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4, 12) == 5
    assert "scratch" in oz.ozaki2_status_string(6)
    assert "gfx950" in oz.ozaki2_status_string(5)


def test_status_strings(L):
    for code in (0, 1, 2, 3, 4, 5, -3):
        assert oz.ozaki2_status_string(code)
    assert oz.ozaki2_set_workspace(0x101, 1024) == -1      # misaligned
    assert oz.ozaki2_set_workspace(None, 0) == 0
    with pytest.raises(oz.Ozaki2Error):
        oz.ozaki2_get_stage_times()                        # nothing timed yet


def test_library_fails_loudly_when_missing(monkeypatch):
    monkeypatch.setattr(oz, "_lib", None)
    monkeypatch.setattr(oz, "LIB_PATH", "/nonexistent/liboz2.so")
    with pytest.raises(ImportError):
        oz.lib()


def test_batched_argument_errors_and_workspace():
    d = 0
    call = oz.ozaki2_dgemm_batched
    one = lambda **kw: dict(dict(transA=["N"], transB=["N"], m=[4], n=[4], k=[4], alpha=[1.0],
                                 A=[d], lda=[4], B=[d], ldb=[4], beta=[0.0], C=[d], ldc=[4],
                                 num_moduli=12), **kw)
    assert call(**one(transA=["X"])) == -2
    assert call(**one(transB=["q"])) == -3
    assert call(**one(m=[-1])) == -4
    assert call(**one(n=[-1])) == -5
    assert call(**one(k=[-1])) == -6
    assert call(**one(lda=[3])) == -9
    assert call(**one(ldb=[3])) == -11
    assert call(**one(ldc=[3])) == -14
    assert call(**one(num_moduli=0)) == -15
    assert call(**one(num_moduli=34)) == -15
    # the second problem is the invalid one
    two = dict(transA=["N", "T"], transB=["N", "N"], m=[4, 4], n=[4, 4], k=[4, 5],
               alpha=[1.0, 1.0], A=[d, d], lda=[4, 4], B=[d, d], ldb=[4, 5], beta=[0.0, 0.0],
               C=[d, d], ldc=[4, 4], num_moduli=12)
    assert call(**two) == -9
    L = oz.lib()
    assert L.ozaki2_dgemm_batched(-1, None, None, None, None, None, None, None, None, None,
                                  None, None, None, None, 12) == -1
    assert L.ozaki2_dgemm_batched(0, None, None, None, None, None, None, None, None, None,
                                  None, None, None, None, 12) == 0
    assert L.ozaki2_dgemm_batched(1, None, None, None, None, None, None, None, None, None,
                                  None, None, None, None, 12) == -2
    # empty outputs only: nothing to do, success without a device
    assert call(**one(m=[0], lda=[1], ldc=[1])) == 0
    # workspace of a batch = sum over problems with a nonempty product of the
    # layout up to the planes plus its plane copies: 4 for a problem of at
    # most 4 output tiles of 256 x 256 and at least 512 padded k (split-K
    # parts), else 1
    ms, ns, ks = [300, 0, 64, 1000, 2000], [200, 5, 64, 17, 1500], [700, 9, 0, 4096, 300]
    pad = lambda x: (x + 255) // 256 * 256
    want = 0
    for a, b, c in zip(ms, ns, ks):
        if a and b and c:
            off, _ = oz.ozaki2_workspace_layout(a, b, c, 12)
            copies = 4 if pad(a) * pad(b) <= 4 * 256 * 256 and pad(c) >= 512 else 1
            want += off[7] + pad(2 * 12 * pad(a) * pad(b) * copies)
    assert oz.ozaki2_workspace_bytes_batched(ms, ns, ks, 12) == want
    assert oz.ozaki2_workspace_bytes_batched([1], [-1], [1], 12) == 0


def test_batched_no_device_on_cpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert oz.ozaki2_dgemm_batched(["N"], ["N"], [4], [4], [4], [1.0], [0], [4], [0], [4],
                                   [0.0], [0], [4], 12) == 5
    assert oz.ozaki2_set_graph(True) == 0 and oz.ozaki2_set_graph(False) == 0
    assert oz.ozaki2_set_autotune(True) == 0 and oz.ozaki2_set_autotune(False) == 0
    assert oz.ozaki2_get_schedule() == -1
    for c in (-1, 0, 5):
        assert oz.ozaki2_set_schedule(c) == 0
    assert oz.ozaki2_set_schedule(6) == -1 and oz.ozaki2_set_schedule(-2) == -1
    assert oz.ozaki2_set_schedule(-1) == 0


def test_mode_setting_host_only():
    # the scaling mode is a per-thread host setting (no device needed)
    assert oz.ozaki2_get_mode() == oz.MODE_ACCURATE
    assert oz.ozaki2_set_mode("fast") == 0 and oz.ozaki2_get_mode() == oz.MODE_FAST
    assert oz.ozaki2_set_mode(2) == -1 and oz.ozaki2_set_mode(-1) == -1
    assert oz.ozaki2_get_mode() == oz.MODE_FAST
    with pytest.raises(ValueError):
        oz.ozaki2_set_mode("fastest")
    assert oz.ozaki2_set_mode(oz.MODE_ACCURATE) == 0 and oz.ozaki2_get_mode() == 0
    # the workspace does not depend on the mode
    oz.ozaki2_set_mode("fast")
    w_fast = oz.ozaki2_workspace_bytes(300, 200, 700, 13)
    oz.ozaki2_set_mode("accurate")
    assert w_fast == oz.ozaki2_workspace_bytes(300, 200, 700, 13)


def test_karatsuba_only_list_host_only():
    # the modulus list is a per-thread host setting; tables, moduli queries
    # and workspace sizes follow it
    assert oz.ozaki2_get_moduli_list() == oz.MODULI_HYBRID
    assert oz.ozaki2_set_moduli_list(5) == -1
    with pytest.raises(ValueError):
        oz.ozaki2_set_moduli_list("binary")
    w_h = oz.ozaki2_workspace_bytes(300, 200, 700, 13)
    assert oz.ozaki2_set_moduli_list("karatsuba") == 0
    try:
        assert oz.ozaki2_get_moduli_list() == oz.MODULI_KARATSUBA
        for N in range(1, 34):
            p, kinds = oz.ozaki2_moduli(N)
            assert p == [q for q, _, _ in ref.moduli_table(N, "karatsuba")]
            assert kinds == [1] * N
            _, pads = oz.ozaki2_workspace_layout(300, 200, 700, N)
            assert pads["M"] == 3 * N
        assert oz.ozaki2_workspace_bytes(300, 200, 700, 13) > w_h
    finally:
        oz.ozaki2_set_moduli_list("hybrid")
    assert oz.ozaki2_workspace_bytes(300, 200, 700, 13) == w_h


def test_int8_list_host_only():
    assert oz.ozaki2_set_moduli_list("int8") == 0
    try:
        assert oz.ozaki2_get_moduli_list() == oz.MODULI_INT8
        for N in range(1, 34):
            p, kinds = oz.ozaki2_moduli(N)
            assert p == [q for q, _, _ in ref.moduli_table(N, "int8")]
            assert kinds == [2] * N
            _, pads = oz.ozaki2_workspace_layout(300, 200, 700, N)
            assert pads["M"] == N
    finally:
        oz.ozaki2_set_moduli_list("hybrid")


def test_blocking_setting_and_workspace():
    assert oz.ozaki2_get_blocking() == (0, 0)
    assert oz.ozaki2_set_blocking(100, 256) == -1
    assert oz.ozaki2_set_blocking(256, -256) == -2
    assert oz.ozaki2_get_blocking() == (0, 0)
    full = oz.ozaki2_workspace_bytes(16384, 16384, 16384, 12)
    assert oz.ozaki2_set_blocking(4096, 4096) == 0
    try:
        assert oz.ozaki2_get_blocking() == (4096, 4096)
        blk = oz.ozaki2_workspace_bytes(16384, 16384, 16384, 12)
        # per-line vectors and bound operands for the whole problem, slices
        # and planes for one 4096 x 4096 block
        M, N, kp = 30, 12, 16384
        lines = 2 * 16384
        want_core = 2 * 16384 * kp + M * 2 * 4096 * kp + 2 * N * 4096 * 4096
        assert want_core < blk < want_core + 64 * lines + 4096
        assert full > 4 * blk
        # a problem that fits one block is not blocked
        assert oz.ozaki2_workspace_bytes(1000, 4000, 300, 12) == \
            oz.ozaki2_workspace_bytes(1000, 4000, 300, 12)
        small = oz.ozaki2_workspace_bytes(1000, 4000, 300, 12)
    finally:
        oz.ozaki2_set_blocking(0, 0)
    assert oz.ozaki2_workspace_bytes(1000, 4000, 300, 12) == small
    assert oz.ozaki2_workspace_bytes(16384, 16384, 16384, 12) == full


def test_workspace_sizes_that_do_not_fit_are_refused():
    # extents above 2^40 and sizes that overflow size_t give 0 (and
    # OZ2_ERR_UNSUPPORTED from ozaki2_dgemm), never a wrapped small size
    ws = oz.ozaki2_workspace_bytes
    assert ws(2 ** 40 + 1, 256, 256, 12) == 0
    assert ws(256, 256, 2 ** 40 + 1, 12) == 0
    assert ws(2 ** 40, 2 ** 40, 256, 12) == 0      # planes: 24 x 2^80 bytes
    assert ws(2 ** 33, 2 ** 33, 256, 12) == 0      # planes: 24 x 2^66 bytes
    big = ws(2 ** 29, 2 ** 29, 2 ** 15, 12)        # about 2^62.6 bytes: fits
    assert big > 2 ** 62
    # k = 2^18 needs 8 k parts of 2^15, each with its own planes: 2^65.6 bytes
    assert ws(2 ** 29, 2 ** 29, 2 ** 18, 12) == 0
    # the sum over a batch must not wrap either
    wb = oz.ozaki2_workspace_bytes_batched
    assert wb([2 ** 29] * 2, [2 ** 29] * 2, [2 ** 15] * 2, 12) == 2 * big
    assert wb([2 ** 29] * 3, [2 ** 29] * 3, [2 ** 15] * 3, 12) == 0
    # ordinary sizes are unchanged: the layout of 8192^3 at N = 12
    assert ws(8192, 8192, 8192, 12) == 5772017920


def test_tensor_wrappers_refuse_bad_operands():
    """dgemm / dgemm_batched check their tensors before any library call: a
    host tensor, another dtype or rank never reaches the kernels."""
    import torch

    a = torch.zeros((4, 3), dtype=torch.float64)
    b = torch.zeros((3, 5), dtype=torch.float64)
    with pytest.raises(TypeError):
        oz.dgemm(a.float(), b)
    with pytest.raises(ValueError, match="2-D"):
        oz.dgemm(a.reshape(-1), b)
    with pytest.raises(ValueError, match="GPU"):
        oz.dgemm(a, b)
    with pytest.raises(TypeError):
        oz.dgemm(a.numpy(), b)
    with pytest.raises(ValueError, match="GPU"):
        oz.dgemm_batched([a], [b])
    with pytest.raises(ValueError, match="as many"):
        oz.dgemm_batched([a, a], [b])
