"""The C ABI's host-side logic (oz2_api.cpp and oz2_tables.cpp) built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, any finding aborts)
against stub kernel launchers, driven through argument checks, workspace
sizes and layouts (plain, blocked, batched, every modulus list, sizes up to
the 2^40 limit and beyond), settings and modulus tables.  Every answer must
equal the real library's (liboz2.so through ctypes) for the same command
sequence."""
import os
import random
import shutil
import subprocess

import pytest

import paper_2603_10634_amd as oz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_10634_amd", "csrc")
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def host_api(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx or not os.path.exists("/opt/rocm/lib/libamdhip64.so"):
        pytest.skip("g++ or the HIP runtime library not available")
    out = str(tmp_path_factory.mktemp("api") / "api_host_check")
    cmd = [gxx, "-O1", "-g", "-std=c++17", *SANITIZE, "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + CSRC, os.path.join(ROOT, "tests", "api_host_check.cpp"),
           os.path.join(CSRC, "oz2_api.cpp"), os.path.join(CSRC, "oz2_tables.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _commands(rng):
    cmds = []
    sizes = [0, 1, 2, 255, 256, 257, 1000, 4096, 8192, 65536, 1 << 18, (1 << 40), (1 << 40) + 1,
             1 << 50, -1]
    for lst in (0, 1, 2):
        cmds.append(("L", lst))
        for blk in ((0, 0), (1024, 1024), (256, 512), (300, 0), (0, -256)):
            cmds.append(("B",) + blk)
            for _ in range(25):
                m, n, k = (rng.choice(sizes) for _ in range(3))
                N = rng.choice([0, 1, 6, 7, 12, 13, 16, 33, 34])
                cmds.append(("W", m, n, k, N))
                cmds.append(("R", m, n, k, N))
            cmds.append(("B", 0, 0))
        for _ in range(25):
            m, n, k = (rng.choice(sizes) for _ in range(3))
            cmds.append(("Y", m, n, k, rng.choice([1, 12, 20, 33, 0])))
        for _ in range(10):
            cnt = rng.randrange(0, 9)
            shp = [(rng.choice(sizes[:10]), rng.choice(sizes[:10]), rng.choice(sizes[:10]))
                   for _ in range(cnt)]
            if rng.random() < 0.2 and shp:
                shp[0] = (5, -3, 7)
            cmds.append(("Q", rng.choice([12, 0, 33]), cnt) + tuple(v for s in shp for v in s))
        for N in (0, 1, 12, 33, 34, 100):
            cmds.append(("P", N))
    cmds.append(("L", 5))
    cmds.append(("L", 0))
    for mode in (0, 1, 2, -1, 0):
        cmds.append(("M", mode))
    for c in (-2, -1, 0, 5, 6, -1):
        cmds.append(("S", c))
    for parts in (-1, 9, 3, 0):
        cmds.append(("K", parts))
        for _ in range(10):
            m, n, k = (rng.choice(sizes) for _ in range(3))
            cmds.append(("W", m, n, k, 12))
            cmds.append(("R", m, n, k, 12))
    for _ in range(200):
        ta, tb = rng.choice("NnTtCcX"), rng.choice("NnTtCcQ")
        m, n, k = (rng.choice([-1, 0, 1, 4, 5, 300]) for _ in range(3))
        lda, ldb, ldc = (rng.choice([0, 1, 3, 4, 5, 300, 301]) for _ in range(3))
        cmds.append(("D", ta, tb, m, n, k, lda, ldb, ldc, rng.choice([0, 1, 12, 33, 34])))
    return cmds


def _library(cmd):
    """The same command through the real library."""
    L = oz.lib()
    op, args = cmd[0], cmd[1:]
    if op == "L":
        return str(L.ozaki2_set_moduli_list(args[0]))
    if op == "B":
        return str(L.ozaki2_set_blocking(*args))
    if op == "M":
        return str(L.ozaki2_set_mode(args[0]))
    if op == "S":
        return str(L.ozaki2_set_schedule(args[0]))
    if op == "K":
        return str(L.ozaki2_set_split(args[0]))
    if op == "W":
        return str(L.ozaki2_workspace_bytes(*args))
    if op == "Y":
        import ctypes
        off = (ctypes.c_int64 * 11)()
        pads = (ctypes.c_int64 * 4)()
        r = L.ozaki2_workspace_layout(*args, off, pads)
        vals = [r] + [off[q] if r > 0 else 0 for q in range(11)] + \
            [pads[q] if r > 0 else 0 for q in range(4)]
        return " ".join(str(v) for v in vals)
    if op == "R":
        import ctypes
        parts, bparts = ctypes.c_int(0), ctypes.c_int(0)
        r = L.ozaki2_workspace_parts(*args, ctypes.byref(parts), ctypes.byref(bparts))
        return f"{r} {parts.value if r == 0 else 0} {bparts.value if r == 0 else 0}"
    if op == "Q":
        N, cnt = args[0], args[1]
        v = args[2:]
        return str(oz.ozaki2_workspace_bytes_batched(list(v[0::3]), list(v[1::3]),
                                                     list(v[2::3]), N) if cnt else
                   L.ozaki2_workspace_bytes_batched(0, None, None, None, N))
    if op == "D":
        ta, tb, m, n, k, lda, ldb, ldc, N = args
        return str(oz.ozaki2_dgemm(ta, tb, m, n, k, 1.0, 0, lda, 0, ldb, 0.0, 0, ldc, N))
    if op == "P":
        import ctypes
        p = (ctypes.c_int32 * 64)()
        kinds = (ctypes.c_int32 * 64)()
        r = L.ozaki2_moduli(args[0], p, kinds)
        return " ".join([str(r)] + ([f"{p[q]}:{kinds[q]}" for q in range(args[0])] if r == 0 else []))
    raise ValueError(op)


def test_host_logic_sanitized_matches_library(host_api):
    import torch
    if torch.cuda.is_available():
        pytest.skip("compares host-only paths; with a GPU present, valid calls would launch")
    rng = random.Random(2603)
    cmds = _commands(rng)
    text = "".join(" ".join(str(v) for v in c) + "\n" for c in cmds)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([host_api], input=text, capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    got = r.stdout.splitlines()
    assert len(got) == len(cmds)
    try:
        want = [_library(c) for c in cmds]
    finally:
        oz.ozaki2_set_moduli_list("hybrid")
        oz.ozaki2_set_blocking(0, 0)
        oz.ozaki2_set_mode("accurate")
        oz.ozaki2_set_schedule(-1)
        oz.ozaki2_set_split(0)
    bad = [(c, g, w) for c, g, w in zip(cmds, got, want) if g != w]
    assert not bad, bad[:5]
