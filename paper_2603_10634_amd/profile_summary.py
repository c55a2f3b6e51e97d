"""Summaries of rocprofv3 runs of bench.py for profiles/.

  python -m paper_2603_10634_amd.profile_summary trace  DIR PREFIX OUT.md  [CMD]
      kernel-trace statistics (PREFIX_kernel_stats.csv) as a markdown table.
  python -m paper_2603_10634_amd.profile_summary counters CSV OUT.md [CMD]
      hardware counters of one rocprofv3 --pmc run (PREFIX_counter_collection.csv),
      mean per dispatch of each kernel, with the derived figures: kernel time
      (from the dispatch timestamps), the clock GRBM_GUI_ACTIVE counted per
      XCD over that time, and MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES over the
      SIMD cycles of the same span (MI355X: 8 XCDs, 256 CUs x 4 SIMDs).
  python -m paper_2603_10634_amd.profile_summary traffic DIR FETCH WRITE OUT.md OUT.json [CMD...]
      HBM bytes per dispatch from a FETCH_SIZE and a WRITE_SIZE counter run
      (FETCH_counter_collection.csv, WRITE_counter_collection.csv), each
      scaled so that the plain 1 GiB device copy that bench.py
      --copy-calibration runs reads exactly 1 GiB fetched and 1 GiB written.
      OUT.json records the residue-product bytes per call (both launches)
      with the SHA-256 of the GEMM source, so bench.py can tell whether the
      counters still describe the built kernel.

The counters report KiB per dispatch; rows are averaged over the dispatches
of each kernel name.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
GEMM_SOURCE = os.path.join(HERE, "csrc", "oz2_gemm.hip")
COPY_BYTES = 1 << 30


def gemm_source_sha() -> str:
    with open(GEMM_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short(name: str) -> str:
    name = name.replace("oz2::(anonymous namespace)::", "").replace("void ", "")
    name = name.split("(")[0]
    return name if len(name) <= 64 else name[:60] + " ..."


def trace(d: str, prefix: str, out: str, cmd: str = "") -> None:
    rows = list(csv.DictReader(open(os.path.join(d, f"{prefix}_kernel_stats.csv"))))
    with open(out, "w") as f:
        f.write(f"# Kernel trace: {os.path.basename(out)}\n\n")
        if cmd:
            f.write(f"Command:\n\n    {cmd}\n\n")
        f.write("| kernel | calls | avg ms | min ms | max ms | % of GPU time |\n|---|---|---|---|---|---|\n")
        for r in rows:
            f.write(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                    f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | "
                    f"{float(r['Percentage']):.2f} |\n")


def _per_kernel(path: str, counter: str):
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[(short(r["Kernel_Name"]), r["Grid_Size"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}


XCDS = 8
SIMDS = 256 * 4


def counters(csv_path: str, out: str, cmd: str = "") -> None:
    vals = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        name = short(r["Kernel_Name"])
        vals[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur[name][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    names = sorted(vals, key=lambda n: -sum(dur[n].values()))
    ctrs = sorted({c for n in vals for c in vals[n]})
    with open(out, "w") as f:
        f.write(f"# Hardware counters per dispatch: {os.path.basename(out)}\n\n")
        if cmd:
            f.write(f"Command:\n\n    {cmd}\n\n")
        f.write("Means over the dispatches of each kernel.  clock = GRBM_GUI_ACTIVE / "
                f"{XCDS} XCDs / kernel time; MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / "
                f"(GRBM_GUI_ACTIVE / {XCDS} x {SIMDS} SIMDs).\n\n")
        f.write("| kernel | dispatches | ms | clock GHz | MFMA busy | "
                + " | ".join(ctrs) + " |\n")
        f.write("|---|---|---|---|---|" + "---|" * len(ctrs) + "\n")
        for n in names:
            d = vals[n]
            t = sum(dur[n].values()) / len(dur[n])
            mean = {c: sum(v) / len(v) for c, v in d.items()}
            grbm = mean.get("GRBM_GUI_ACTIVE")
            clock = f"{grbm / XCDS / t / 1e9:.2f}" if grbm and t > 0 else ""
            mfma = mean.get("SQ_VALU_MFMA_BUSY_CYCLES")
            busy = f"{100 * mfma / (grbm / XCDS * SIMDS):.1f} %" if grbm and mfma else ""
            f.write(f"| `{n}` | {len(dur[n])} | {t * 1e3:.3f} | {clock} | {busy} | "
                    + " | ".join(f"{mean[c]:.4g}" if c in mean else "" for c in ctrs) + " |\n")


def traffic(d: str, fetch: str, write: str, out_md: str, out_json: str, cmd: str = "") -> None:
    fk = _per_kernel(os.path.join(d, f"{fetch}_counter_collection.csv"), "FETCH_SIZE")
    wk = _per_kernel(os.path.join(d, f"{write}_counter_collection.csv"), "WRITE_SIZE")
    # the calibration copy: the copy kernel dispatches that wrote 1 GiB
    copy_w = [v for (n, g), v in wk.items() if "copyBuffer" in n and abs(v * 1024 - COPY_BYTES) < 0.01 * COPY_BYTES]
    copy_f = [v for (n, g), v in fk.items() if "copyBuffer" in n and v * 1024 > 0.25 * COPY_BYTES]
    if not copy_w or not copy_f:
        raise SystemExit("no calibration copy found (run bench.py with --copy-calibration)")
    fscale = COPY_BYTES / (max(copy_f) * 1024)
    wscale = COPY_BYTES / (max(copy_w) * 1024)
    keys = sorted(set(fk) | set(wk), key=lambda k: -(fk.get(k, 0) + wk.get(k, 0)))
    gemm = {"fetch": 0.0, "write": 0.0}
    with open(out_md, "w") as f:
        f.write(f"# HBM traffic per dispatch: {os.path.basename(out_md)}\n\n")
        if cmd:
            f.write("Commands:\n\n" + "".join(f"    {c}\n" for c in cmd.split(" ;; ")) + "\n")
        f.write(f"Scale factors from the 1 GiB copy: FETCH_SIZE x {fscale:.4f}, "
                f"WRITE_SIZE x {wscale:.4f}.\n\n")
        f.write("| kernel | grid | fetched MB | written MB |\n|---|---|---|---|\n")
        for k in keys:
            fb = fk.get(k, 0.0) * 1024 * fscale
            wb = wk.get(k, 0.0) * 1024 * wscale
            if fb + wb < 1e6:
                continue
            f.write(f"| `{k[0]}` | {k[1]} | {fb / 1e6:.1f} | {wb / 1e6:.1f} |\n")
            if k[0].startswith("k_residue_gemm"):
                gemm["fetch"] += fb
                gemm["write"] += wb
    rec = {"kernel": "residue products (square and Karatsuba launches of one call)",
           "fetch_bytes_per_call": gemm["fetch"], "write_bytes_per_call": gemm["write"],
           "bytes_per_call": gemm["fetch"] + gemm["write"], "fetch_scale": fscale,
           "write_scale": wscale, "gemm_source_sha256": gemm_source_sha(), "commands": cmd}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "trace":
        trace(a[1], a[2], a[3], " ".join(a[4:]))
    elif a and a[0] == "counters":
        counters(a[1], a[2], " ".join(a[3:]))
    elif a and a[0] == "traffic":
        traffic(a[1], a[2], a[3], a[4], a[5], " ".join(a[6:]))
    else:
        print(__doc__)
        sys.exit(2)
