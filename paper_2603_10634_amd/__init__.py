"""MI355X (gfx950) FP8 Ozaki-II DGEMM emulation: Python binding.

A thin ctypes layer over liboz2.so, whose C ABI is declared in
include/ozaki2.h.  Every function here only marshals arguments; all of the
arithmetic runs in the library's HIP kernels.  Device memory and streams come
from PyTorch.  There is no fallback: if the library is not built, or no
gfx950 GPU is current, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

__all__ = [
    "Ozaki2Error", "lib", "ozaki2_dgemm", "ozaki2_workspace_bytes", "ozaki2_set_stream",
    "ozaki2_set_workspace", "ozaki2_set_timing", "ozaki2_get_stage_times",
    "ozaki2_get_kernel_times", "ozaki2_moduli", "ozaki2_workspace_layout",
    "ozaki2_workspace_parts", "ozaki2_release", "ozaki2_status_string", "ozaki2_dgemm_batched", "ozaki2_workspace_bytes_batched",
    "ozaki2_set_graph", "ozaki2_set_autotune", "ozaki2_get_schedule", "ozaki2_set_schedule",
    "ozaki2_set_split", "ozaki2_set_mode", "ozaki2_get_mode", "MODE_ACCURATE", "MODE_FAST", "ozaki2_set_moduli_list",
    "ozaki2_get_moduli_list", "MODULI_HYBRID", "MODULI_KARATSUBA", "MODULI_INT8",
    "ozaki2_set_blocking", "ozaki2_get_blocking", "dgemm", "dgemm_batched",
    "LIB_PATH", "HEADER_PATH", "header_functions", "ozaki2_dgemm_noalloc",
    "NOALLOC_SCRATCH_BYTES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboz2.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ozaki2.h")

MODE_ACCURATE = 0   # OZ2_MODE_ACCURATE
MODE_FAST = 1       # OZ2_MODE_FAST
MODULI_HYBRID = 0     # OZ2_MODULI_HYBRID
MODULI_KARATSUBA = 1  # OZ2_MODULI_KARATSUBA
MODULI_INT8 = 2       # OZ2_MODULI_INT8

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_p64 = ctypes.POINTER(ctypes.c_int64)
_pd = ctypes.POINTER(ctypes.c_double)
_pvp = ctypes.POINTER(ctypes.c_void_p)


class Ozaki2Error(RuntimeError):
    """A nonzero status returned by the library."""

    def __init__(self, func: str, status: int):
        self.status = status
        super().__init__(f"{func} returned {status}: {ozaki2_status_string(status)}")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded liboz2.so (loaded on first use)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_2603_10634_amd.build` "
            "(hipcc, gfx950) first")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "ozaki2_dgemm": (ctypes.c_int, [ctypes.c_char, ctypes.c_char, _i64, _i64, _i64,
                                        ctypes.c_double, _vp, _i64, _vp, _i64,
                                        ctypes.c_double, _vp, _i64, ctypes.c_int]),
        "ozaki2_workspace_bytes": (ctypes.c_size_t, [_i64, _i64, _i64, ctypes.c_int]),
        "ozaki2_set_stream": (ctypes.c_int, [_vp]),
        "ozaki2_set_workspace": (ctypes.c_int, [_vp, ctypes.c_size_t]),
        "ozaki2_set_timing": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_get_stage_times": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float)]),
        "ozaki2_get_kernel_times": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
        "ozaki2_moduli": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]),
        "ozaki2_workspace_layout": (ctypes.c_int, [_i64, _i64, _i64, ctypes.c_int,
                                                   ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "ozaki2_workspace_parts": (ctypes.c_int, [_i64, _i64, _i64, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_int)]),
        "ozaki2_release": (ctypes.c_int, []),
        "ozaki2_dgemm_batched": (ctypes.c_int, [ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p,
                                                _p64, _p64, _p64, _pd, _pvp, _p64, _pvp, _p64,
                                                _pd, _pvp, _p64, ctypes.c_int]),
        "ozaki2_workspace_bytes_batched": (ctypes.c_size_t, [ctypes.c_int, _p64, _p64, _p64,
                                                             ctypes.c_int]),
        "ozaki2_set_graph": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_set_autotune": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_get_schedule": (ctypes.c_int, []),
        "ozaki2_set_schedule": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_set_split": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_set_mode": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_get_mode": (ctypes.c_int, []),
        "ozaki2_set_moduli_list": (ctypes.c_int, [ctypes.c_int]),
        "ozaki2_get_moduli_list": (ctypes.c_int, []),
        "ozaki2_set_blocking": (ctypes.c_int, [_i64, _i64]),
        "ozaki2_get_blocking": (ctypes.c_int, [_p64, _p64]),
        "ozaki2_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "ozaki2_dgemm_noalloc": (ctypes.c_int, [ctypes.c_char, ctypes.c_char, _i64, _i64, _i64,
                                                ctypes.c_double, _vp, _i64, _vp, _i64,
                                                ctypes.c_double, _vp, _i64, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions declared in include/ozaki2.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ozaki2_\w+)\s*\(", text)))


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _ch(c: str) -> bytes:
    return c.encode() if isinstance(c, str) else bytes([c])


def ozaki2_status_string(status: int) -> str:
    return lib().ozaki2_status_string(int(status)).decode()


def ozaki2_dgemm(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                 num_moduli) -> int:
    """Column-major C <- alpha op(A) op(B) + beta C (see include/ozaki2.h).
    A, B, C are device pointers (int) or tensors; returns the status code."""
    return lib().ozaki2_dgemm(_ch(transA), _ch(transB), m, n, k, float(alpha), _ptr(A), lda,
                              _ptr(B), ldb, float(beta), _ptr(C), ldc, int(num_moduli))


def ozaki2_dgemm_noalloc(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                         num_moduli) -> int:
    """ozaki2_dgemm on the library's fixed scratch buffer, for callers that
    cannot allocate (see include/ozaki2.h); returns the status code."""
    return lib().ozaki2_dgemm_noalloc(_ch(transA), _ch(transB), m, n, k, float(alpha), _ptr(A),
                                      lda, _ptr(B), ldb, float(beta), _ptr(C), ldc,
                                      int(num_moduli))


NOALLOC_SCRATCH_BYTES = 256 << 20   # OZ2_NOALLOC_SCRATCH_BYTES


def ozaki2_workspace_bytes(m, n, k, num_moduli) -> int:
    return lib().ozaki2_workspace_bytes(m, n, k, num_moduli)


def ozaki2_set_stream(stream) -> int:
    """stream: a torch.cuda.Stream, a raw hipStream_t (int) or None."""
    raw = getattr(stream, "cuda_stream", stream)
    return lib().ozaki2_set_stream(raw or None)


def ozaki2_set_workspace(ptr, nbytes: int) -> int:
    return lib().ozaki2_set_workspace(_ptr(ptr) or None, nbytes)


def ozaki2_set_timing(on: bool) -> int:
    return lib().ozaki2_set_timing(1 if on else 0)


def ozaki2_get_stage_times() -> list[float]:
    """[quant, gemms, requant, dequant, others] milliseconds of the last timed call."""
    buf = (ctypes.c_float * 5)()
    st = lib().ozaki2_get_stage_times(buf)
    if st != 0:
        raise Ozaki2Error("ozaki2_get_stage_times", st)
    return list(buf)


def ozaki2_get_kernel_times() -> list[float]:
    """Per-kernel-group milliseconds of the last timed call (6 entries)."""
    buf = (ctypes.c_float * 6)()
    r = lib().ozaki2_get_kernel_times(buf, 6)
    if r < 0:
        raise Ozaki2Error("ozaki2_get_kernel_times", -r)
    return list(buf)[:r]


def ozaki2_moduli(num_moduli: int) -> tuple[list[int], list[int]]:
    p = (ctypes.c_int32 * num_moduli)()
    kinds = (ctypes.c_int32 * num_moduli)()
    if lib().ozaki2_moduli(num_moduli, p, kinds) != 0:
        raise ValueError(f"invalid number of moduli {num_moduli}")
    return list(p), list(kinds)


def ozaki2_workspace_layout(m, n, k, num_moduli) -> tuple[list[int], dict]:
    off = (_i64 * 11)()
    pads = (_i64 * 4)()
    r = lib().ozaki2_workspace_layout(m, n, k, num_moduli, off, pads)
    if r < 0:
        raise ValueError("invalid sizes")
    return list(off)[:r], dict(mp=pads[0], np=pads[1], kp=pads[2], M=pads[3])


def ozaki2_workspace_parts(m, n, k, num_moduli) -> tuple[int, int]:
    """(k parts of the residue products = plane copies, k parts of the bound
    product) of an ozaki2_dgemm call of this shape under the thread's
    settings."""
    parts, bparts = ctypes.c_int(0), ctypes.c_int(0)
    if lib().ozaki2_workspace_parts(m, n, k, num_moduli, ctypes.byref(parts),
                                    ctypes.byref(bparts)) < 0:
        raise ValueError("invalid sizes")
    return parts.value, bparts.value


def ozaki2_release() -> int:
    return lib().ozaki2_release()


def _arr(ctype, values):
    values = list(values)
    return (ctype * max(1, len(values)))(*values)


def ozaki2_dgemm_batched(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                         num_moduli) -> int:
    """Batched column-major DGEMMs (see include/ozaki2.h).  Every argument but
    num_moduli is a sequence with one entry per problem; A, B, C entries are
    device pointers (int) or tensors.  Returns the status code."""
    count = len(m)
    if any(len(x) != count for x in (transA, transB, n, k, alpha, A, lda, B, ldb, beta, C, ldc)):
        raise ValueError("batched arguments differ in length")
    ta = b"".join(_ch(c) for c in transA) + b"\0"
    tb = b"".join(_ch(c) for c in transB) + b"\0"
    return lib().ozaki2_dgemm_batched(
        count, ta, tb, _arr(ctypes.c_int64, m), _arr(ctypes.c_int64, n),
        _arr(ctypes.c_int64, k), _arr(ctypes.c_double, [float(x) for x in alpha]),
        _arr(ctypes.c_void_p, [_ptr(x) or None for x in A]), _arr(ctypes.c_int64, lda),
        _arr(ctypes.c_void_p, [_ptr(x) or None for x in B]), _arr(ctypes.c_int64, ldb),
        _arr(ctypes.c_double, [float(x) for x in beta]),
        _arr(ctypes.c_void_p, [_ptr(x) or None for x in C]), _arr(ctypes.c_int64, ldc),
        int(num_moduli))


def ozaki2_workspace_bytes_batched(m, n, k, num_moduli) -> int:
    return lib().ozaki2_workspace_bytes_batched(len(m), _arr(ctypes.c_int64, m),
                                                _arr(ctypes.c_int64, n),
                                                _arr(ctypes.c_int64, k), num_moduli)


def ozaki2_set_graph(on: bool) -> int:
    return lib().ozaki2_set_graph(1 if on else 0)


def ozaki2_set_autotune(on: bool) -> int:
    return lib().ozaki2_set_autotune(1 if on else 0)


def ozaki2_get_schedule() -> int:
    return lib().ozaki2_get_schedule()


def ozaki2_set_schedule(config: int) -> int:
    """Force the batched residue-product configuration (0..5), or -1 for the
    default / autotuned one."""
    return lib().ozaki2_set_schedule(int(config))


def ozaki2_set_split(parts: int) -> int:
    """Force the number of k parts (1..8) of the calling thread's
    ozaki2_dgemm residue products, or 0 for the library's rule."""
    return lib().ozaki2_set_split(int(parts))


def _mode_code(mode) -> int:
    if isinstance(mode, str):
        codes = {"accurate": MODE_ACCURATE, "fast": MODE_FAST}
        if mode not in codes:
            raise ValueError("mode must be 'accurate' or 'fast'")
        return codes[mode]
    return int(mode)


def ozaki2_set_mode(mode) -> int:
    """mode: MODE_ACCURATE / MODE_FAST, or 'accurate' / 'fast'."""
    return lib().ozaki2_set_mode(_mode_code(mode))


def ozaki2_get_mode() -> int:
    return lib().ozaki2_get_mode()


def _list_code(moduli) -> int:
    if isinstance(moduli, str):
        codes = {"hybrid": MODULI_HYBRID, "karatsuba": MODULI_KARATSUBA, "int8": MODULI_INT8}
        if moduli not in codes:
            raise ValueError("moduli list must be 'hybrid', 'karatsuba' or 'int8'")
        return codes[moduli]
    return int(moduli)


def ozaki2_set_moduli_list(moduli) -> int:
    """moduli: MODULI_HYBRID / MODULI_KARATSUBA / MODULI_INT8, or 'hybrid' /
    'karatsuba' / 'int8'."""
    return lib().ozaki2_set_moduli_list(_list_code(moduli))


def ozaki2_get_moduli_list() -> int:
    return lib().ozaki2_get_moduli_list()


def ozaki2_set_blocking(m_blk: int, n_blk: int) -> int:
    return lib().ozaki2_set_blocking(m_blk, n_blk)


def ozaki2_get_blocking() -> tuple[int, int]:
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    lib().ozaki2_get_blocking(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def _check_tensor(name: str, t, device) -> None:
    """Marshalling checks of the tensor wrappers: a 2-D float64 tensor in GPU
    memory on `device` (device pointers are all the library accepts; a host
    pointer handed to its kernels would fault the GPU)."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, not {t.dtype}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D, not {t.dim()}-D")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor, not on {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the other operands on {device}")


class _ModeScope:
    """Sets the calling thread's mode for one call and restores it after."""

    def __init__(self, mode):
        self.mode = mode

    def __enter__(self):
        self.prev = ozaki2_get_mode()
        if self.mode is not None:
            st = ozaki2_set_mode(self.mode)
            if st != 0:
                raise Ozaki2Error("ozaki2_set_mode", st)

    def __exit__(self, *exc):
        ozaki2_set_mode(self.prev)
        return False


def dgemm_batched(As, Bs, num_moduli: int = 12, mode=None):
    """Row-major C_q = A_q B_q for lists of 2-D float64 CUDA tensors, as one
    batched call on torch's current stream; returns the list of C_q.  `mode`
    ('accurate' / 'fast', default: the thread's setting) applies to this call."""
    import torch

    As, Bs = list(As), list(Bs)
    if len(As) != len(Bs):
        raise ValueError("dgemm_batched takes as many A as B tensors")
    dev = As[0].device if As else None
    for a, b in zip(As, Bs):
        _check_tensor("A", a, dev)
        _check_tensor("B", b, dev)
    As = [a.contiguous() for a in As]
    Bs = [b.contiguous() for b in Bs]
    Cs, args = [], []
    for a, b in zip(As, Bs):
        m, k = a.shape
        if b.shape[0] != k:
            raise ValueError("inner dimensions differ")
        n = b.shape[1]
        c = torch.empty((m, n), dtype=torch.float64, device=a.device)
        Cs.append(c)
        args.append((n, m, k, b, max(1, n), a, max(1, k), c, max(1, n)))
    if not args:
        return Cs
    ozaki2_set_stream(torch.cuda.current_stream(dev))
    with torch.cuda.device(dev), _ModeScope(mode):
        st = ozaki2_dgemm_batched(["N"] * len(args), ["N"] * len(args), [x[0] for x in args],
                                  [x[1] for x in args], [x[2] for x in args], [1.0] * len(args),
                                  [x[3] for x in args], [x[4] for x in args],
                                  [x[5] for x in args], [x[6] for x in args], [0.0] * len(args),
                                  [x[7] for x in args], [x[8] for x in args], num_moduli)
    if st != 0:
        raise Ozaki2Error("ozaki2_dgemm_batched", st)
    return Cs


def dgemm(A, B, num_moduli: int = 12, alpha: float = 1.0, beta: float = 0.0, C=None,
          mode=None):
    """Row-major C = alpha A B + beta C for 2-D float64 CUDA tensors (via the
    column-major identity C^T = B^T A^T).  Runs on torch's current stream.
    `mode` ('accurate' / 'fast', default: the thread's setting) applies to
    this call."""
    import torch

    _check_tensor("A", A, A.device if isinstance(A, torch.Tensor) else None)
    _check_tensor("B", B, A.device)
    A = A.contiguous()
    B = B.contiguous()
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = torch.empty((m, n), dtype=torch.float64, device=A.device)
        beta = 0.0
    else:
        # the library writes m x n doubles at C with leading dimension n:
        # anything smaller, strided or elsewhere is refused before the call
        _check_tensor("C", C, A.device)
        if tuple(C.shape) != (m, n):
            raise ValueError(f"C has shape {tuple(C.shape)}, expected {(m, n)}")
        if not C.is_contiguous():
            raise ValueError("C must be contiguous (it is written in place)")
    ozaki2_set_stream(torch.cuda.current_stream(A.device))
    with torch.cuda.device(A.device), _ModeScope(mode):
        st = ozaki2_dgemm("N", "N", n, m, k, alpha, B, max(1, n), A, max(1, k), beta, C,
                          max(1, n), num_moduli)
    if st != 0:
        raise Ozaki2Error("ozaki2_dgemm", st)
    return C
