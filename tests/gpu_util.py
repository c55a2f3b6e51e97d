"""Helpers for the GPU tests: run the library through its C ABI on seeded
inputs and read back the output and the intermediate buffers of the
workspace."""
from __future__ import annotations

import numpy as np
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import to_colmajor, from_colmajor
from workloads.reference import dd_dot_rows, normalised_error


def device():
    return torch.device("cuda", 0)


class Run:
    """Output of one ozaki2_dgemm call."""

    def __init__(self, status, C, ldc, m, n, ws=None, off=None, pads=None, parts=1):
        self.status = status
        self.Cbuf = C
        self.ldc = ldc
        self.C = from_colmajor(C, m, n, ldc) if status == 0 and m and n else None
        self.ws = ws
        self.off = off
        self.pads = pads
        self.parts = parts  # k parts of the residue products: plane copies
        self.m, self.n = m, n

    # ---- workspace views (see ozaki2_workspace_layout) ----
    def _vec(self, idx, dtype, count):
        o = self.off[idx]
        return np.frombuffer(self.ws[o:o + count * np.dtype(dtype).itemsize].tobytes(), dtype=dtype)

    def lines(self, idx, dtype=np.int32):
        mp, np_ = self.pads["mp"], self.pads["np"]
        v = self._vec(idx, dtype, mp + np_)
        return v[:self.m], v[mp:mp + self.n]

    def fixups(self):
        """Number of lines whose scale exponent was settled by the exact fix-up."""
        return int(self._vec(10, np.uint32, 2).sum())

    @staticmethod
    def _unblock(buf, rows, kp):
        """rows x kp view of a k-blocked buffer: element (r, h) at
        (h // 64) * 64 rows + 64 r + h % 64."""
        return buf.reshape(kp // 64, rows, 64).transpose(1, 0, 2).reshape(rows, kp)

    def bar(self, which):
        mp, np_, kp = self.pads["mp"], self.pads["np"], self.pads["kp"]
        rows = mp if which == "A" else np_
        o = self.off[3 if which == "A" else 4]
        return self._unblock(self.ws[o:o + rows * kp], rows, kp)

    def slices(self, which):
        mp, np_, kp, M = self.pads["mp"], self.pads["np"], self.pads["kp"], self.pads["M"]
        rows = mp if which == "A" else np_
        o = self.off[5 if which == "A" else 6]
        return np.stack([self._unblock(self.ws[o + q * rows * kp:o + (q + 1) * rows * kp], rows, kp)
                         for q in range(M)])

    def planes(self, N, ps):
        """C'_l for the moduli ps: the sum of the plane copies of the k parts
        reduced to smod(., p_l)."""
        mp, np_ = self.pads["mp"], self.pads["np"]
        o = self.off[7]
        size = 2 * N * mp * np_
        copies = self.parts
        assert copies >= 1 and o + copies * size <= len(self.ws)
        parts = np.frombuffer(self.ws[o:o + copies * size].tobytes(),
                              dtype=np.int16).reshape(copies, N, np_, mp).astype(np.int64)
        total = parts.sum(axis=0)
        if copies == 1:
            return total
        h = np.array([p // 2 for p in ps], dtype=np.int64)[:, None, None]
        return (total + h) % np.array(ps, dtype=np.int64)[:, None, None] - h


def run(opA, opB, N, transA="N", transB="N", alpha=1.0, beta=0.0, Cin=None,
        pad=(0, 0, 0), keep_ws=False, stream=None, mode="accurate", moduli="hybrid",
        blocking=(0, 0)):
    """Column-major ozaki2_dgemm on op(A) (m x k) and op(B) (k x n) given as
    numpy arrays, in the given scaling mode and modulus list; leading-dimension
    padding is filled with NaN (A, B) or 7.0 (C) so reads or writes outside
    the views show.  `blocking` = (m_blk, n_blk) runs the call m/n-blocked."""
    m, k = opA.shape
    n = opB.shape[1]
    Ab, lda = to_colmajor(opA, transA, ld=(max(1, m) if transA in "Nn" else max(1, k)) + pad[0])
    Bb, ldb = to_colmajor(opB, transB, ld=(max(1, k) if transB in "Nn" else max(1, n)) + pad[1])
    ldc = max(1, m) + pad[2]
    Cmat = np.zeros((m, n)) if Cin is None else Cin
    Cb, _ = to_colmajor(Cmat, "N", ld=ldc, fill=7.0)
    dev = device()
    tA = torch.from_numpy(Ab.copy()).to(dev)
    tB = torch.from_numpy(Bb.copy()).to(dev)
    tC = torch.from_numpy(Cb.copy()).to(dev)
    assert oz.ozaki2_set_moduli_list(moduli) == 0
    assert oz.ozaki2_set_blocking(*blocking) == 0
    try:
        return _run_list(tA, tB, tC, transA, transB, m, n, k, alpha, lda, ldb, beta, ldc, N,
                         keep_ws, stream, mode, dev)
    finally:
        oz.ozaki2_set_moduli_list("hybrid")
        oz.ozaki2_set_blocking(0, 0)


def _run_list(tA, tB, tC, transA, transB, m, n, k, alpha, lda, ldb, beta, ldc, N, keep_ws,
              stream, mode, dev):
    wbytes = oz.ozaki2_workspace_bytes(m, n, k, N)
    ws = torch.full((wbytes + 256,), 0xEE, dtype=torch.uint8, device=dev)
    base = (ws.data_ptr() + 255) // 256 * 256
    oz.ozaki2_set_workspace(base, wbytes)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    oz.ozaki2_set_stream(s)
    assert oz.ozaki2_set_mode(mode) == 0
    try:
        st = oz.ozaki2_dgemm(transA, transB, m, n, k, alpha, tA, lda, tB, ldb, beta, tC, ldc, N)
        torch.cuda.synchronize(dev)
    finally:
        oz.ozaki2_set_workspace(None, 0)
        oz.ozaki2_set_mode("accurate")
    off = pads = None
    wsh = None
    parts = 1
    if keep_ws:
        # keep_ws == "lines": only the per-line vectors, which precede Abar
        off, pads = oz.ozaki2_workspace_layout(m, n, k, N)
        parts = oz.ozaki2_workspace_parts(m, n, k, N)[0]
        shift = base - ws.data_ptr()
        upto = off[3] if keep_ws == "lines" else wbytes
        wsh = ws[shift:shift + upto].cpu().numpy()
    return Run(st, tC.cpu().numpy(), ldc, m, n, wsh, off, pads, parts)


def check_stages(r: Run, opA, opB, N, st=None, mode="accurate", moduli="hybrid"):
    """Every stored intermediate equals the oracle's, bit for bit.  Fast mode
    stores no bound operands; there every line is flagged as finalized from
    its exact bound and no line is queued for a fix-up."""
    if st is None:
        _, st = ref.emulate(opA, opB, N, keep_stages=True, mode=mode, moduli_set=moduli)
    m, k = opA.shape
    n = opB.shape[1]
    EA, EB = r.lines(1)
    assert np.array_equal(EA, st["EA"]) and np.array_equal(EB, st["EB"]), "ufp exponents"
    eA, eB = r.lines(2)
    assert np.array_equal(eA, st["e"]) and np.array_equal(eB, st["f"]), "scale exponents"
    sA, sB = r.lines(0)
    assert np.array_equal(sA, st["sA"]) and np.array_equal(sB, st["sB"]), "shifts"
    if mode == "fast":
        fA, fB = r.lines(9, np.uint32)
        assert np.all(fA & 4) and np.all(fB & 4), "fast mode: every line from its norm"
        assert r.fixups() == 0, "fast mode queues no fix-ups"
    else:
        Ab = r.bar("A")
        Bb = r.bar("B")
        assert np.array_equal(Ab[:m, :k], ref.e4m3_encode_exact(st["Abar"])), "Abar"
        assert np.array_equal(Bb[:n, :k], ref.e4m3_encode_exact(st["Bbar"].T)), "Bbar"
        assert not Ab[m:].any() and not Ab[:, k:].any(), "Abar padding"
        assert not Bb[n:].any() and not Bb[:, k:].any(), "Bbar padding"
    SA = r.slices("A")
    SB = r.slices("B")
    sl = 0
    for pm in st["per_modulus"]:
        # FP8 digits as E4M3 codes; INT8 residues as two's-complement bytes
        enc = ((lambda x: x.astype(np.int8).view(np.uint8)) if pm["kind"] == "int8"
               else ref.e4m3_encode_exact)
        for dA, dB in zip(pm["dA"], pm["dB"]):
            assert np.array_equal(SA[sl, :m, :k], enc(dA)), f"A slice {sl}"
            assert np.array_equal(SB[sl, :n, :k], enc(dB.T)), f"B slice {sl}"
            assert not SA[sl, m:].any() and not SA[sl, :, k:].any(), f"A slice {sl} padding"
            assert not SB[sl, n:].any() and not SB[sl, :, k:].any(), f"B slice {sl} padding"
            sl += 1
    assert sl == r.pads["M"]
    P = r.planes(N, [pm["p"] for pm in st["per_modulus"]])
    for l, plane in enumerate(st["planes"]):
        assert np.array_equal(P[l, :n, :m].T.astype(np.int64), plane), f"plane {l}"


class split:
    """Context: the calling thread's ozaki2_dgemm calls use `parts` k parts
    for their residue products (0: the library's rule)."""

    def __init__(self, parts):
        self.parts = parts

    def __enter__(self):
        assert oz.ozaki2_set_split(self.parts) == 0

    def __exit__(self, *exc):
        oz.ozaki2_set_split(0)


def same_bits(a, b):
    """Bitwise equality, NaN matching NaN."""
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


def sample_lines(n, count, seed, extra=()):
    """The edge lines 0, 1, n/2, n-2, n-1, `count` seeded others and `extra`."""
    rng = np.random.default_rng(seed)
    fixed = [0, 1, n // 2, n - 2, n - 1]
    return np.unique(np.concatenate([fixed, rng.integers(0, n, count), list(extra)]).astype(np.int64))


def sweep_sample(m, n, cancel=False):
    """The rows and columns the accuracy sweep (accuracy_sweep) measures its
    error on: first, middle, last and five seeded rows (all when m <= 128;
    the cancellation block's rows 1, 100, 255 with it) and the first 1024
    columns."""
    if m <= 128:
        rows = np.arange(m)
    else:
        rng = np.random.default_rng(m)
        rows = np.unique(np.concatenate([[0, m // 2, m - 1], rng.integers(0, m, 5)]))
        if cancel:
            rows = np.unique(np.concatenate([rows, [1, 100, 255]]))
    return rows.astype(np.int64), np.arange(min(n, 1024), dtype=np.int64)


def check_sampled(A, B, N, rows, cols, transA="N", transB="N", mode="accurate",
                  moduli="hybrid", cache=None, err_rows=None, err_cols=None, err_max=1e-15,
                  label=""):
    """One library call on op(A) x op(B) stored as transA / transB; the shifts
    of the sampled lines and the outputs rows x cols bit for bit against the
    oracle (line-restricted scaling), and the normalised error on
    err_rows x err_cols (a subset of the sample; default: all of it).
    `cache` (a dict, returned) keeps the oracle's bounds, results and
    double-double reference for further calls on the same logical inputs."""
    print(f"{label}: GPU N={N} {moduli} {mode} {transA}{transB}", flush=True)
    r = run(A, B, N, transA, transB, keep_ws="lines", mode=mode, moduli=moduli)
    assert r.status == 0
    cache = {} if cache is None else cache
    if ("bounds", mode) not in cache:
        print(f"{label}: oracle bounds", flush=True)
        cache[("bounds", mode)] = ref.line_bounds(
            A, B, rows, cols, mode, log=lambda msg: print(f"{label}: oracle {msg}", flush=True))
    key = (N, moduli, mode)
    if key not in cache:
        sc = ref.scaling_from_bounds(cache[("bounds", mode)], N, moduli)
        print(f"{label}: oracle products", flush=True)
        cache[key] = (sc, ref.products(sc, slice(None), slice(None))[0])
    sc, want = cache[key]
    sA, sB = r.lines(0)
    assert np.array_equal(sA[rows], sc["sA"]), "shifts of the sampled rows"
    assert np.array_equal(sB[cols], sc["sB"]), "shifts of the sampled columns"
    got = r.C[np.ix_(rows, cols)]
    assert same_bits(got, want), f"{int(np.sum(got.view(np.int64) != want.view(np.int64)))} outputs differ"
    er = rows if err_rows is None else np.asarray(err_rows)
    ec = cols if err_cols is None else np.asarray(err_cols)
    if "dd" not in cache:
        cache["dd"] = dd_dot_rows(A[er], B[:, ec])
    hi, lo = cache["dd"]
    sub = got[np.ix_(np.searchsorted(rows, er), np.searchsorted(cols, ec))]
    err = normalised_error(sub, hi, lo, np.abs(A[er]), np.abs(B[:, ec]))
    print(f"{label}: N={N} normalised error {err:.3e}, exact fix-ups {r.fixups()}",
          flush=True)
    assert err <= err_max, err
    return cache
