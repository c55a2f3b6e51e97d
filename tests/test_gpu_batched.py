"""Batched calls (grouped launches over uneven problems, the residue products
of the whole batch in one persistent launch), graph capture, the residue
product configurations (tile program, split-K) and the autotuner, through the
C ABI.

A batched call must give, for every problem, exactly the C that a separate
ozaki2_dgemm call gives (which the parity tests pin to the oracle), and the
problems are also compared with the oracle directly (small ones in full,
large ones on sampled outputs)."""
import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import batch_shapes, config_seed, phi_matrix, to_colmajor, from_colmajor

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda", 0)


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    ok = both_nan | (a.view(np.int64) == b.view(np.int64))
    if not ok.all():
        bad = np.argwhere(~ok)
        i = tuple(bad[0])
        print(f"  {len(bad)} of {a.size} entries differ; first at {i}: {a[i]!r} vs {b[i]!r}",
              flush=True)
    return bool(ok.all())


class Batch:
    """Device buffers of a batch of column-major problems built from seeded
    op(A), op(B) (numpy) with the given storage transposes."""

    def __init__(self, shapes, seed, trans=None, alpha=None, beta=None, phi=1.0):
        self.shapes = shapes
        cnt = len(shapes)
        self.trans = trans or [("N", "N")] * cnt
        self.alpha = alpha or [1.0] * cnt
        self.beta = beta or [0.0] * cnt
        self.opA, self.opB, self.Cin = [], [], []
        self.tA, self.tB, self.tC0 = [], [], []
        self.lda, self.ldb, self.ldc = [], [], []
        for q, (m, n, k) in enumerate(shapes):
            ta, tb = self.trans[q]
            A = phi_matrix(m, k, phi, seed + 2 * q)
            B = phi_matrix(k, n, phi, seed + 2 * q + 1)
            Cin = phi_matrix(m, n, 1.0, seed + 100000 + q)
            Ab, lda = to_colmajor(A, ta, ld=(max(1, m) if ta == "N" else max(1, k)) + q % 3)
            Bb, ldb = to_colmajor(B, tb, ld=(max(1, k) if tb == "N" else max(1, n)) + q % 2)
            Cb, ldc = to_colmajor(Cin, "N", ld=max(1, m) + q % 4, fill=7.0)
            self.opA.append(A)
            self.opB.append(B)
            self.Cin.append(Cin)
            self.tA.append(torch.from_numpy(Ab.copy()).to(dev()))
            self.tB.append(torch.from_numpy(Bb.copy()).to(dev()))
            self.tC0.append(torch.from_numpy(Cb.copy()).to(dev()))
            self.lda.append(lda)
            self.ldb.append(ldb)
            self.ldc.append(ldc)

    def fresh_C(self):
        return [c.clone() for c in self.tC0]

    def batched(self, N, Cs):
        m = [s[0] for s in self.shapes]
        n = [s[1] for s in self.shapes]
        k = [s[2] for s in self.shapes]
        return oz.ozaki2_dgemm_batched([t[0] for t in self.trans], [t[1] for t in self.trans],
                                       m, n, k, self.alpha, self.tA, self.lda, self.tB,
                                       self.ldb, self.beta, Cs, self.ldc, N)

    def singles(self, N, Cs):
        for q, (m, n, k) in enumerate(self.shapes):
            st = oz.ozaki2_dgemm(self.trans[q][0], self.trans[q][1], m, n, k, self.alpha[q],
                                 self.tA[q], self.lda[q], self.tB[q], self.ldb[q],
                                 self.beta[q], Cs[q], self.ldc[q], N)
            assert st == 0, (q, st)

    def host(self, Cs):
        torch.cuda.synchronize()
        return [c.cpu().numpy() for c in Cs]


def _pad(x):
    return (x + 255) // 256 * 256


def _split_copies(m, n, k, N):
    """Bytes of the three extra residue-plane copies a batched problem holds
    when split-K may apply to it (at most 4 tiles, padded k >= 512)."""
    if _pad(m) * _pad(n) <= 4 * 256 * 256 and _pad(k) >= 512:
        return 3 * 2 * N * _pad(m) * _pad(n)
    return 0


def _setup():
    oz.ozaki2_set_stream(torch.cuda.current_stream(dev()))
    oz.ozaki2_set_workspace(None, 0)
    oz.ozaki2_set_graph(False)
    oz.ozaki2_set_autotune(False)
    oz.ozaki2_set_schedule(-1)


def _uneven(count, lo, hi, seed):
    shapes = batch_shapes(count, lo, hi, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    trans = [(("N", "T")[rng.integers(2)], ("N", "T")[rng.integers(2)]) for _ in shapes]
    alpha = [float(x) for x in rng.choice([1.0, -0.5, 2.0], size=count)]
    beta = [float(x) for x in rng.choice([0.0, 0.0, 1.0, -1.5], size=count)]
    return shapes, trans, alpha, beta


def test_batched_equals_single_calls_and_oracle():
    _setup()
    shapes, trans, alpha, beta = _uneven(14, 1, 600, config_seed(4, 1))
    # degenerate members: empty output, k = 0, alpha = 0
    shapes += [(0, 17, 5), (33, 0, 9), (40, 21, 0), (25, 30, 12)]
    trans += [("N", "N")] * 4
    alpha += [1.0, 1.0, 1.5, 0.0]
    beta += [0.0, 1.0, -2.0, 0.5]
    print(f"batched parity: {shapes}", flush=True)
    b = Batch(shapes, config_seed(4, 2), trans, alpha, beta)
    for N in (12, 7):
        Cb = b.fresh_C()
        assert b.batched(N, Cb) == 0
        Cs = b.fresh_C()
        b.singles(N, Cs)
        hb, hs = b.host(Cb), b.host(Cs)
        for q in range(len(shapes)):
            assert _same(hb[q], hs[q]), (N, q, shapes[q])
        # direct oracle comparison on the small members
        for q, (m, n, k) in enumerate(shapes):
            if m * n * k == 0 or m * n * k > 4e6:
                continue
            Chat = ref.emulate(b.opA[q], b.opB[q], N)
            want = ref.combine_alpha_beta(Chat, alpha[q], beta[q], b.Cin[q])
            got = from_colmajor(hb[q], m, n, b.ldc[q])
            assert _same(got, want), (N, q, shapes[q])
        # the padding of C beyond each problem's m rows is untouched
        for q, (m, n, k) in enumerate(shapes):
            if n and b.ldc[q] > m:
                pad = hb[q].reshape(-1)[: n * b.ldc[q]].reshape(n, b.ldc[q])[:, m:]
                assert np.all(pad == 7.0), q


def test_batched_sub_batches_with_small_workspace():
    _setup()
    shapes, trans, alpha, beta = _uneven(9, 20, 700, config_seed(4, 3))
    b = Batch(shapes, config_seed(4, 4), trans, alpha, beta)
    N = 12
    need = [oz.ozaki2_workspace_bytes(m, n, k, N) + _split_copies(m, n, k, N)
            for m, n, k in shapes]
    total = oz.ozaki2_workspace_bytes_batched([s[0] for s in shapes], [s[1] for s in shapes],
                                              [s[2] for s in shapes], N)
    assert total == sum(need)
    # room for the largest problem plus a little: several sub-batches
    cap = max(need) + min(need)
    ws = torch.empty(cap + 256, dtype=torch.uint8, device=dev())
    base = (ws.data_ptr() + 255) // 256 * 256
    print(f"sub-batches: workspace {cap} of {total}", flush=True)
    Cs = b.fresh_C()
    b.singles(N, Cs)
    oz.ozaki2_set_workspace(base, cap)
    try:
        Cb = b.fresh_C()
        assert b.batched(N, Cb) == 0
    finally:
        oz.ozaki2_set_workspace(None, 0)
    hb, hs = b.host(Cb), b.host(Cs)
    for q in range(len(shapes)):
        assert _same(hb[q], hs[q]), q


def test_batched_workspace_too_small_is_an_error():
    _setup()
    shapes = [(300, 200, 100), (64, 64, 64)]
    b = Batch(shapes, config_seed(4, 5))
    need = max(oz.ozaki2_workspace_bytes(m, n, k, 12) for m, n, k in shapes)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev())
    base = (ws.data_ptr() + 255) // 256 * 256
    oz.ozaki2_set_workspace(base, need - 256)
    try:
        assert b.batched(12, b.fresh_C()) == 3     # OZ2_ERR_WORKSPACE
    finally:
        oz.ozaki2_set_workspace(None, 0)


@pytest.mark.parametrize("which", ["batched", "single"])
def test_graph_replays_follow_new_data(which):
    """Graph mode: the first call captures, later calls with the same
    arguments replay; new data written into the same buffers between replays,
    and eager work in between, must show up exactly as in eager calls."""
    _setup()
    shapes = [(300, 257, 190), (64, 700, 33), (129, 65, 513)] if which == "batched" \
        else [(333, 280, 400)]
    b = Batch(shapes, config_seed(4, 6), beta=[0.5] * len(shapes))
    N = 12
    Cg = b.fresh_C()        # the same output buffers at every replay
    for rep in range(4):
        print(f"graph {which} replay {rep}", flush=True)
        if rep:
            # new input values in the same buffers
            for q, t in enumerate(b.tA):
                t.mul_(-1.5 if rep % 2 else 0.25)
        for c, c0 in zip(Cg, b.tC0):
            c.copy_(c0)
        Ce = b.fresh_C()
        oz.ozaki2_set_graph(True)
        try:
            if which == "batched":
                assert b.batched(N, Cg) == 0
            else:
                b.singles(N, Cg)
        finally:
            oz.ozaki2_set_graph(False)
        # eager work on the stream between replays
        junk = torch.ones(1 << 20, device=dev()).sum()
        torch.cuda.synchronize()
        if which == "batched":
            assert b.batched(N, Ce) == 0
        else:
            b.singles(N, Ce)
        hg, he = b.host(Cg), b.host(Ce)
        for q in range(len(shapes)):
            assert _same(hg[q], he[q]), (rep, q)
        assert junk.item() == float(1 << 20)
    # a graph replayed with a different C pointer is a different argument list
    Cg2 = b.fresh_C()
    oz.ozaki2_set_graph(True)
    try:
        if which == "batched":
            assert b.batched(N, Cg2) == 0
        else:
            b.singles(N, Cg2)
    finally:
        oz.ozaki2_set_graph(False)
    for q, (x, y) in enumerate(zip(b.host(Cg2), b.host(Ce))):
        assert _same(x, y), q


def test_autotuner_picks_a_schedule_and_keeps_results():
    _setup()
    shapes, trans, alpha, beta = _uneven(10, 64, 1500, config_seed(4, 7))
    b = Batch(shapes, config_seed(4, 8), trans, alpha, beta)
    N = 12
    C0 = b.fresh_C()
    assert b.batched(N, C0) == 0
    assert oz.ozaki2_get_schedule() == 0
    oz.ozaki2_set_autotune(True)
    try:
        C1 = b.fresh_C()
        assert b.batched(N, C1) == 0
        s1 = oz.ozaki2_get_schedule()
        C2 = b.fresh_C()
        assert b.batched(N, C2) == 0
        assert oz.ozaki2_get_schedule() == s1
    finally:
        oz.ozaki2_set_autotune(False)
    print(f"autotuned configuration {s1}", flush=True)
    assert 0 <= s1 < 6
    h0, h1, h2 = b.host(C0), b.host(C1), b.host(C2)
    for q in range(len(shapes)):
        assert _same(h0[q], h1[q]) and _same(h0[q], h2[q]), q


@pytest.mark.parametrize("N,moduli", [(12, "hybrid"), (14, "int8")])
def test_every_configuration_same_bits(N, moduli):
    """Both tile programs and every split-K limit give the C of per-problem
    calls, on problems that split (few tiles, long k, one of them beyond a k
    chunk of 2^15) and problems that do not; forced configurations replay
    from graphs too."""
    _setup()
    shapes = [(64, 64, 4096), (300, 200, 2000), (256, 512, 1024), (1000, 900, 800),
              (70, 90, 40000), (33, 17, 300), (512, 512, 256)]
    trans = [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T"), ("N", "N"), ("T", "T"), ("N", "N")]
    b = Batch(shapes, config_seed(4, 9), trans, beta=[0.0, 1.0, -0.5, 0.0, 2.0, 0.0, 0.25])
    assert oz.ozaki2_set_moduli_list(moduli) == 0
    try:
        Cs = b.fresh_C()
        b.singles(N, Cs)
        hs = b.host(Cs)
        for c in range(6):
            print(f"configuration {c} ({moduli})", flush=True)
            assert oz.ozaki2_set_schedule(c) == 0
            for graph in (False, True):
                oz.ozaki2_set_graph(graph)
                Cb = b.fresh_C()
                assert b.batched(N, Cb) == 0
                assert oz.ozaki2_get_schedule() == c
                hb = b.host(Cb)
                for q in range(len(shapes)):
                    assert _same(hb[q], hs[q]), (c, graph, q, shapes[q])
            oz.ozaki2_set_graph(False)
        # the smallest members against the oracle directly
        for q in (5, 0):
            m, n, k = shapes[q]
            Chat = ref.emulate(b.opA[q], b.opB[q], N, moduli_set=moduli)
            want = ref.combine_alpha_beta(Chat, 1.0, b.beta[q], b.Cin[q])
            assert _same(from_colmajor(hs[q], m, n, b.ldc[q]), want), q
    finally:
        oz.ozaki2_set_schedule(-1)
        oz.ozaki2_set_graph(False)
        oz.ozaki2_set_moduli_list("hybrid")


def test_autotune_cache_file(tmp_path):
    """The autotuner's choice is written to the file named by
    OZ2_AUTOTUNE_CACHE in the documented form (read back here as JSON); a
    later process with tuning off takes that choice for the same shape
    bucket, and one whose file is corrupt falls back to the default."""
    import json
    import os
    import subprocess
    import sys
    path = tmp_path / "tune.json"
    code = (
        "import sys, torch, paper_2603_10634_amd as oz\n"
        "sys.path.insert(0, 'tests')\n"
        "from test_gpu_batched import Batch, _uneven\n"
        "from workloads import config_seed\n"
        "oz.ozaki2_set_stream(torch.cuda.current_stream())\n"
        "shapes, trans, alpha, beta = _uneven(6, 64, 900, config_seed(4, 11))\n"
        "b = Batch(shapes, config_seed(4, 12), trans, alpha, beta)\n"
        "oz.ozaki2_set_autotune(sys.argv[1] == 'tune')\n"
        "assert b.batched(12, b.fresh_C()) == 0\n"
        "torch.cuda.synchronize()\n"
        "print('CONFIG', oz.ozaki2_get_schedule())\n")
    env = dict(os.environ, OZ2_AUTOTUNE_CACHE=str(path))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def child(arg):
        print(f"cache file: child process ({arg})", flush=True)
        r = subprocess.run([sys.executable, "-c", code, arg], cwd=root, env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return int(r.stdout.split("CONFIG")[1].split()[0])

    chosen = child("tune")
    doc = json.loads(path.read_text())
    assert doc["oz2_autotune"] == 1 and len(doc["entries"]) == 1
    entry = doc["entries"][0]
    assert entry["config"] == chosen and entry["key"].startswith("n12m0l0:")
    # another configuration recorded for the bucket: a fresh process uses it
    other = (chosen + 1) % 6
    path.write_text(path.read_text().replace(f'"config": {chosen}', f'"config": {other}'))
    assert child("run") == other
    # a malformed file is ignored: the default configuration
    path.write_text('{"oz2_autotune": 1, "entries": [\n{"key": "x", "config": 99}\n]}\n')
    assert child("run") == 0


def test_batched_many_uneven_problems_sampled():
    """512 problems with m, n, k log-uniform in [64, 4096] (inputs drawn on the
    GPU from a seeded generator): on a sample of 48 problems the batched call
    equals per-problem calls and the oracle on sampled outputs; the autotuned
    configuration gives the same bits for every problem."""
    _setup()
    shapes = batch_shapes(512, 64, 4096, config_seed(4, 0))
    g = torch.Generator(device=dev())
    g.manual_seed(config_seed(4, 0))
    tA, tB, tC = [], [], []
    for (m, n, k) in shapes:
        a = (torch.rand((k, m), generator=g, device=dev(), dtype=torch.float64) - 0.5) * \
            torch.exp(torch.randn((k, m), generator=g, device=dev(), dtype=torch.float64))
        bb = (torch.rand((n, k), generator=g, device=dev(), dtype=torch.float64) - 0.5) * \
            torch.exp(torch.randn((n, k), generator=g, device=dev(), dtype=torch.float64))
        tA.append(a)
        tB.append(bb)
        tC.append(torch.empty((n, m), dtype=torch.float64, device=dev()))
    cnt = len(shapes)
    m = [s[0] for s in shapes]
    n = [s[1] for s in shapes]
    k = [s[2] for s in shapes]
    args = lambda Cs: (["N"] * cnt, ["N"] * cnt, m, n, k, [1.0] * cnt, tA, m, tB, k,
                       [0.0] * cnt, Cs, m, 12)
    print("512-problem batch", flush=True)
    assert oz.ozaki2_dgemm_batched(*args(tC)) == 0
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(5))
    sample = sorted(rng.choice(cnt, size=48, replace=False).tolist())
    for q in sample:
        c = torch.empty_like(tC[q])
        assert oz.ozaki2_dgemm("N", "N", m[q], n[q], k[q], 1.0, tA[q], m[q], tB[q], k[q], 0.0,
                               c, m[q], 12) == 0
        torch.cuda.synchronize()
        assert torch.equal(c.view(torch.int64), tC[q].view(torch.int64)), q
        # the oracle directly, on sampled outputs (their lines' exponents
        # from the whole problem's bound product)
        opA = tA[q].cpu().numpy().T           # m x k
        opB = tB[q].cpu().numpy().T           # k x n
        rows = np.unique(np.concatenate([[0, m[q] - 1], rng.integers(0, m[q], 4)]))
        cols = np.unique(np.concatenate([[0, n[q] - 1], rng.integers(0, n[q], 4)]))
        sc = ref.scaling_lines(opA, opB, 12, rows, cols)
        want, _ = ref.products(sc, slice(None), slice(None))
        got = tC[q].cpu().numpy().T[np.ix_(rows, cols)]
        assert _same(got, want), (q, shapes[q])
    oz.ozaki2_set_autotune(True)
    try:
        tC2 = [torch.empty_like(c) for c in tC]
        assert oz.ozaki2_dgemm_batched(*args(tC2)) == 0
        torch.cuda.synchronize()
        print(f"512-problem batch: schedule {oz.ozaki2_get_schedule()}", flush=True)
    finally:
        oz.ozaki2_set_autotune(False)
    for q in range(cnt):
        assert torch.equal(tC2[q].view(torch.int64), tC[q].view(torch.int64)), q
