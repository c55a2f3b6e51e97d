"""Normalised error of the emulated DGEMM against the number of moduli.

    python -m paper_2603_10634_amd.accuracy_sweep --size 4096 --phi 0.5 2 4 \
        --moduli 2 20 [--mode accurate|fast] [--moduli-list hybrid|karatsuba|int8] \
        [--shape M N K] [--normal] [--cancel] [--out FILE.md]

For each phi (entries (U - 1/2) exp(phi N(0,1)), the paper's test matrices,
seeded as workload --config numbers them; --normal: standard-normal entries
instead) and each N, one call of the
library on op(A) (M x K) times op(B) (K x N), both stored column-major; the
error max |C - AB| / (|A| |B|) is taken over sampled rows (first, middle,
last and five seeded others; all rows when M <= 128) and the first 1024
columns against a double-double reference.  --cancel makes rows 0..255 of
op(A) orthogonal to columns 0..255 of op(B) up to a 1e-8 perturbation (the
large stress workload's cancellation block) and samples them too.  One line
per case is printed as it completes, then the smallest N whose error is at
most the target for each phi; --out also writes the table as markdown.
"""
from __future__ import annotations

import argparse
import sys
import time


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=4096, help="m = n = k (unless --shape)")
    ap.add_argument("--shape", type=int, nargs=3, default=None, metavar=("M", "N", "K"))
    ap.add_argument("--phi", type=float, nargs="+", default=[0.5, 2.0, 4.0])
    ap.add_argument("--normal", action="store_true", help="standard-normal entries")
    ap.add_argument("--cancel", action="store_true", help="add the cancellation block")
    ap.add_argument("--config", type=int, default=2, help="seed group of the workload")
    ap.add_argument("--moduli", type=int, nargs=2, default=[2, 20], metavar=("FIRST", "LAST"))
    ap.add_argument("--mode", choices=["accurate", "fast"], default="accurate")
    ap.add_argument("--moduli-list", choices=["hybrid", "karatsuba", "int8"], default="hybrid")
    ap.add_argument("--target", type=float, default=1e-15)
    ap.add_argument("--out", type=str, default=None, help="markdown file for the table")
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2603_10634_amd as oz
    from workloads import cancellation_block, config_seed, normal_matrix, phi_matrix, phi_seed
    from workloads.reference import dd_dot_rows, normalised_error

    m, n, k = args.shape if args.shape else (args.size,) * 3
    dev = torch.device("cuda", 0)
    oz.ozaki2_set_stream(torch.cuda.current_stream(dev))
    if oz.ozaki2_set_mode(args.mode) != 0 or oz.ozaki2_set_moduli_list(args.moduli_list) != 0:
        raise RuntimeError("invalid mode or moduli list")
    rng = np.random.default_rng(m)
    if m <= 128:
        rows = np.arange(m)
    else:
        rows = np.unique(np.concatenate([[0, m // 2, m - 1], rng.integers(0, m, 5)]))
        if args.cancel:
            rows = np.unique(np.concatenate([rows, [1, 100, 255]]))
    cols = np.arange(min(n, 1024))
    dists = ["normal"] if args.normal else args.phi
    Ns = list(range(args.moduli[0], args.moduli[1] + 1))
    table = {}
    nmin = {}
    for q, phi in enumerate(dists):
        seed = config_seed(args.config, q) if phi == "normal" else phi_seed(args.config, phi)
        if phi == "normal":
            A = normal_matrix(m, k, seed)
            B = normal_matrix(k, n, seed + 1)
        else:
            A = phi_matrix(m, k, phi, seed)
            B = phi_matrix(k, n, phi, seed + 1)
        if args.cancel:
            A = cancellation_block(A, B, min(256, m), min(256, n), 1e-8, seed + 2)
        hi, lo = dd_dot_rows(A[rows], B[:, cols])
        absA, absB = np.abs(A[rows]), np.abs(B[:, cols])
        tA = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev)   # m x k, lda = m
        tB = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)   # k x n, ldb = k
        tC = torch.empty((n, m), dtype=torch.float64, device=dev)
        trows = torch.from_numpy(rows).to(dev)
        del A, B
        for N in Ns:
            st = oz.ozaki2_dgemm("N", "N", m, n, k, 1.0, tA, m, tB, k, 0.0, tC, m, N)
            if st != 0:
                raise oz.Ozaki2Error("ozaki2_dgemm", st)
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            oz.ozaki2_dgemm("N", "N", m, n, k, 1.0, tA, m, tB, k, 0.0, tC, m, N)
            torch.cuda.synchronize(dev)
            ms = (time.perf_counter() - t0) * 1e3
            C = tC[:, trows].cpu().numpy().T[:, cols]
            err = normalised_error(C, hi, lo, absA, absB)
            table[(phi, N)] = (err, ms)
            if err <= args.target and phi not in nmin:
                nmin[phi] = N
            print(f"shape={m}x{n}x{k} phi={phi} N={N} mode={args.mode} list={args.moduli_list} "
                  f"error={err:.3e} ms={ms:.2f}", flush=True)
        del tA, tB, tC
        oz.ozaki2_release()
    for phi in dists:
        print(f"shape={m}x{n}x{k} phi={phi}: smallest N with error <= {args.target:g}: "
              f"{nmin.get(phi, 'none in range')}", flush=True)
    if args.out:
        dname = "standard normal" if args.normal else "(U - 1/2) exp(phi N(0,1))"
        with open(args.out, "w") as f:
            f.write(f"# Normalised error against the number of moduli: {m} x {n} x {k}\n\n")
            f.write("Command:\n\n    python -m paper_2603_10634_amd.accuracy_sweep "
                    + " ".join(sys.argv[1:]) + "\n\n")
            f.write(f"Entries {dname}{', with the cancellation block' if args.cancel else ''}; "
                    f"{args.mode} mode, {args.moduli_list} moduli; error = max |C - AB| / "
                    f"(|A||B|) over {len(rows)} rows x {len(cols)} columns against a "
                    "double-double reference; time = one call, synchronised.\n\n")
            f.write("| N | " + " | ".join(f"phi = {p}" if p != "normal" else "normal"
                                          for p in dists) + " |\n")
            f.write("|---|" + "---|" * len(dists) + "\n")
            for N in Ns:
                cells = [f"{table[(p, N)][0]:.2e} ({table[(p, N)][1]:.1f} ms)" for p in dists]
                f.write(f"| {N} | " + " | ".join(cells) + " |\n")
            f.write(f"\nSmallest N with error <= {args.target:g}: "
                    + ", ".join(f"{'phi = ' + str(p) if p != 'normal' else 'normal'}: "
                                f"{nmin.get(p, 'none in range')}" for p in dists) + "\n")


if __name__ == "__main__":
    main()
