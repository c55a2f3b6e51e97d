"""The large-scale stress workload at its full size: m = n = k = 16384,
entries (U - 0.5) exp(phi N(0,1)) with phi = 1 and a mixed-sign cancellation
block (rows 0..255 of op(A) orthogonal to columns 0..255 of op(B) up to a 1e-8
perturbation), through the FP8 hybrid path and the INT8 arm in fast mode at
their full-accuracy moduli counts (13 and 16, the paper's fast-mode counts).
Sampled outputs (inside and outside the cancellation block) are compared bit
for bit with the oracle, and the normalised error of each arm is checked
against a double-double reference."""
import time

import numpy as np
import pytest
import torch

import paper_2603_10634_amd as oz
from oracle import ozaki2_ref as ref
from workloads import phi_matrix, config_seed, cancellation_block
from workloads.reference import dd_dot_rows, normalised_error

pytestmark = pytest.mark.gpu


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.int64) == b.view(np.int64))))


def test_large_cancellation_both_arms():
    n = 16384
    s = config_seed(5, 0)
    print("large: generating", flush=True)
    A = phi_matrix(n, n, 1.0, s)
    B = phi_matrix(n, n, 1.0, s + 1)
    A = cancellation_block(A, B, 256, 256, 1e-8, s + 2)
    dev = torch.device("cuda", 0)
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    rows = np.array([0, 1, 200, 255, 9000, 16383])
    cols = np.concatenate([np.arange(0, 256, 5), np.array([4097, 16383])])
    hi, lo = dd_dot_rows(A[rows], B[:, cols])
    for moduli, N in (("int8", 16), ("hybrid", 13)):
        print(f"large: GPU {moduli} N={N} fast", flush=True)
        assert oz.ozaki2_set_moduli_list(moduli) == 0
        try:
            C = oz.dgemm(tA, tB, N, mode="fast")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C = oz.dgemm(tA, tB, N, mode="fast")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            Cs = C[torch.from_numpy(rows).to(dev)][:, torch.from_numpy(cols).to(dev)].cpu().numpy()
            del C
        finally:
            oz.ozaki2_set_moduli_list("hybrid")
            oz.ozaki2_release()
        print(f"large: {moduli} N={N}: {dt * 1e3:.1f} ms, {2 * n ** 3 / dt / 1e12:.1f} TFLOP/s",
              flush=True)
        print(f"large: oracle {moduli}", flush=True)
        sc = ref.scaling(A, B, N, mode="fast", moduli_set=moduli)
        want, _ = ref.products(sc, rows, cols)
        del sc
        assert _same(Cs, want), moduli
        err = normalised_error(Cs, hi, lo, np.abs(A[rows]), np.abs(B[:, cols]))
        print(f"large: {moduli} N={N} normalised error {err:.3e}", flush=True)
        assert err <= 1e-15, (moduli, err)
