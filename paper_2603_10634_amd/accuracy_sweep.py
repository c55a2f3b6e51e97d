"""Normalised error of the emulated DGEMM against the number of moduli.

    python -m paper_2603_10634_amd.accuracy_sweep --size 4096 --phi 0.5 2 4 \
        --moduli 2 20 [--mode accurate|fast] [--moduli-list hybrid|karatsuba|int8]

For each phi (entries (U - 1/2) exp(phi N(0,1)), the paper's test matrices)
and each N, one call of the library on m = n = k = size; the error
max |C - AB| / (|A| |B|) is taken over sampled rows (first, middle, last and
five seeded others) and the first 1024 columns against a double-double
reference.  One line per case is printed as it completes, then the smallest
N whose error is at most 1e-15 for each phi.
"""
from __future__ import annotations

import argparse
import time


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--phi", type=float, nargs="+", default=[0.5, 2.0, 4.0])
    ap.add_argument("--moduli", type=int, nargs=2, default=[2, 20], metavar=("FIRST", "LAST"))
    ap.add_argument("--mode", choices=["accurate", "fast"], default="accurate")
    ap.add_argument("--moduli-list", choices=["hybrid", "karatsuba", "int8"], default="hybrid")
    ap.add_argument("--target", type=float, default=1e-15)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2603_10634_amd as oz
    from workloads import config_seed, phi_matrix
    from workloads.reference import dd_dot_rows, normalised_error

    n = args.size
    dev = torch.device("cuda", 0)
    oz.ozaki2_set_stream(torch.cuda.current_stream(dev))
    if oz.ozaki2_set_mode(args.mode) != 0 or oz.ozaki2_set_moduli_list(args.moduli_list) != 0:
        raise RuntimeError("invalid mode or moduli list")
    rng = np.random.default_rng(n)
    rows = np.unique(np.concatenate([[0, n // 2, n - 1], rng.integers(0, n, 5)]))
    cols = np.arange(min(n, 1024))
    nmin = {}
    for q, phi in enumerate(args.phi):
        seed = config_seed(2, q)
        A = phi_matrix(n, n, phi, seed)
        B = phi_matrix(n, n, phi, seed + 1)
        hi, lo = dd_dot_rows(A[rows], B[:, cols])
        absA, absB = np.abs(A[rows]), np.abs(B[:, cols])
        tA = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev)
        tB = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
        tC = torch.empty((n, n), dtype=torch.float64, device=dev)
        for N in range(args.moduli[0], args.moduli[1] + 1):
            st = oz.ozaki2_dgemm("N", "N", n, n, n, 1.0, tA, n, tB, n, 0.0, tC, n, N)
            if st != 0:
                raise oz.Ozaki2Error("ozaki2_dgemm", st)
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            oz.ozaki2_dgemm("N", "N", n, n, n, 1.0, tA, n, tB, n, 0.0, tC, n, N)
            torch.cuda.synchronize(dev)
            ms = (time.perf_counter() - t0) * 1e3
            C = tC[:, torch.from_numpy(rows).to(dev)].cpu().numpy().T[:, cols]
            err = normalised_error(C, hi, lo, absA, absB)
            if err <= args.target and phi not in nmin:
                nmin[phi] = N
            print(f"size={n} phi={phi} N={N} mode={args.mode} list={args.moduli_list} "
                  f"error={err:.3e} ms={ms:.2f}", flush=True)
        del tA, tB, tC
        oz.ozaki2_release()
    for phi in args.phi:
        print(f"size={n} phi={phi}: smallest N with error <= {args.target:g}: "
              f"{nmin.get(phi, 'none in range')}", flush=True)


if __name__ == "__main__":
    main()
