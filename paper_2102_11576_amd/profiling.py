"""Summaries of rocprofv3 output for the kernels of librsfde.

    python -m paper_2102_11576_amd.profiling stats  <kernel_stats.csv>
    python -m paper_2102_11576_amd.profiling counters <fetch counter_collection.csv>
        <write counter_collection.csv> --n1 N1 --n2 N2 --out <file>

`stats` aggregates rocprofv3 --kernel-trace --stats rows by kernel family (all
template instances of one kernel together), so that the average launch
duration is comparable with bench.py's event timing.  `counters` turns two
--pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
`bench.py --mode kernels` into measured HBM bytes per family, scaled by what
the same counters read for the run's plain 256 MiB device copy, and writes a
small JSON text file (with a hash of the kernel sources) that bench.py reads
to fill roofline.traffic.
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# kernel-name pattern -> family used by rsfde_profile_read
FAMILIES = [
    (r"k_multidot<", "multidot"),
    (r"k_axpy_givens<", "axpy_givens"),
    (r"k_update<", "update"),
    (r"k_mv_rows<", "mv_rows"),
    (r"k_mv_cols<", "mv_cols"),
    (r"k_(pc|sd)_rows_fwd<", "pc_rows_fwd"),
    (r"k_(pc|sd)_cols<", "pc_cols"),
    (r"k_(pc|sd)_rows_inv<", "pc_rows_inv"),
    (r"k_(pc|sd)_rows_inv_mv<", "pc_inv_mv_rows"),
    (r"k_dst_cols<", "dst_cols"),
    (r"k_gemm_bf16", "pc_gemm_bf16"),
    (r"k_residual\b", "residual"),
    (r"k_rhs\b", "rhs"),
    (r"k_dot\b", "dot"),
    (r"k_bgram<", "block_gram"),
    (r"k_bupd<", "block_update"),
    (r"k_cd_rows_fwd<", "cd_rows_fwd"),
    (r"k_cd_cols<", "cd_cols"),
    (r"k_cd_rows_inv<", "cd_rows_inv"),
    (r"k_scale_copy", "other"),
]

# One-block finishing kernels launched right after a streaming kernel belong
# to its step (rsfde_profile brackets both): their time goes to the parent
# family, their launches are not counted again.
FINISHERS = [
    (r"k_multidot_finish", "multidot"),
    (r"k_givens", "axpy_givens"),
    (r"k_residual_finish", "residual"),
    (r"k_rhs_finish", "rhs"),
    (r"k_dot_finish", "dot"),
    (r"k_bgram_finish", "block_gram"),
]


def finisher_parent(name: str):
    for pat, fam in FINISHERS:
        if re.search(pat, name):
            return fam
    return None


def family(name: str) -> str:
    p = finisher_parent(name)
    if p:
        return p
    for pat, fam in FAMILIES:
        if re.search(pat, name):
            suffix = ""
            m = re.search(r"<(double|float)", name)
            if m and (fam.startswith("pc_") or fam.startswith("cd_") or fam == "dst_cols"):
                suffix = "<" + m.group(1) + ">"
            return fam + suffix
    return "other"


def source_hash() -> str:
    h = hashlib.sha256()
    for fn in sorted(os.listdir(CSRC)):
        if fn.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(fn.encode())
            h.update(open(os.path.join(CSRC, fn), "rb").read())
    return h.hexdigest()[:16]


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        f = family(r["Name"])
        if not finisher_parent(r["Name"]):
            agg[f][0] += int(r["Calls"])
        agg[f][1] += float(r["TotalDurationNs"])
    tot = sum(v[1] for v in agg.values())
    lines = [f"{'family':16s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'share':>6s}"]
    for f, (c, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{f:16s} {c:7d} {ns / 1e6:10.2f} {ns / c / 1e3:9.2f} {100 * ns / tot:5.1f}%")
    return "\n".join(lines)


def _alg_bytes(name: str, n1: int, n2: int) -> float:
    """Algorithmic bytes of one launch (each operand read once, result written once)."""
    N, S = n1 * n2, (n1 + 1) * n2
    m = re.search(r"k_multidot<(\d+)>", name)
    if m:
        return 8.0 * (int(m.group(1)) + 1) * N
    m = re.search(r"k_axpy_givens<(\d+), true>", name)
    if m:
        return 8.0 * (int(m.group(1)) + 2) * N
    m = re.search(r"k_update<(\d+)>", name)
    if m:
        return 8.0 * (int(m.group(1)) + 2) * N
    if "k_mv_rows<" in name:
        return 17.0 * N
    if "k_mv_cols<" in name:
        return 24.0 * N
    ts = 8.0 if "<double" in name else 4.0
    if re.search(r"k_(pc|sd)_rows_fwd<", name):
        return 8.0 * N + ts * S
    if re.search(r"k_(pc|sd)_cols<", name):
        return 3.0 * ts * S
    if re.search(r"k_(pc|sd)_rows_inv<", name):
        return 2.0 * ts * S + 9.0 * N
    if re.search(r"k_(pc|sd)_rows_inv_mv<", name):  # with the s-step shift term read (sub)
        return 2.0 * ts * S + 25.0 * N
    return 0.0


def counters(fetch_csv: str, write_csv: str, n1: int, n2: int, copy_bytes: float) -> dict:
    def load(path, counter):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                d[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
        return d
    fe, wr = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    # calibration: the largest copy kernel of the run moved copy_bytes each way
    cf = [k for k in fe if "copyBuffer" in k]
    if not cf:
        raise SystemExit("no copy kernel in the counter run")
    fetch_copy = max(max(fe[k]) for k in cf)
    write_copy = max(max(wr.get(k, [0.0])) for k in cf)
    kf, kw = copy_bytes / fetch_copy, copy_bytes / write_copy
    fam = collections.defaultdict(lambda: [0.0, 0.0, 0.0, 0])
    for k in fe:
        f = family(k)
        if f == "other" or finisher_parent(k):
            continue
        alg = _alg_bytes(k, n1, n2)
        if alg <= 0:
            continue
        n = min(len(fe[k]), len(wr.get(k, [])))
        for i in range(n):
            fam[f][0] += fe[k][i] * kf
            fam[f][1] += wr[k][i] * kw
            fam[f][2] += alg
            fam[f][3] += 1
    out = {"source_hash": source_hash(), "n1": n1, "n2": n2,
           "calibration": {"copy_bytes": copy_bytes, "fetch_factor": kf, "write_factor": kw},
           "families": {}}
    for f, (fb, wb, ab, n) in fam.items():
        out["families"][f] = {"launches": n, "fetch_bytes_avg": fb / n, "write_bytes_avg": wb / n,
                              "alg_bytes_avg": ab / n, "traffic_over_alg": (fb + wb) / ab}
    return out


def sq_summary(csv_paths) -> str:
    """Per-family sums of SQ counters (one or more --pmc runs), divided by the
    launch count: instruction mix, VALU and LDS activity and LDS bank
    conflicts of each kernel family."""
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            f = family(r["Kernel_Name"])
            if finisher_parent(r["Kernel_Name"]):
                continue
            vals[f][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[f].add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
    names = sorted({c for f in vals for c in vals[f]})
    lines = ["family           " + " ".join(f"{n[3:]:>20s}" for n in names) + "  (per launch)"]
    for f in sorted(vals, key=lambda k: -vals[k].get("SQ_BUSY_CYCLES", 0.0)):
        n = max(1, len(disp[f]))
        lines.append(f"{f:16s} " + " ".join(f"{vals[f].get(c, 0.0) / n:20.4g}" for c in names))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    b = sub.add_parser("counters")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--n1", type=int, required=True)
    b.add_argument("--n2", type=int, required=True)
    b.add_argument("--copy-bytes", type=float, default=256.0 * 1024 * 1024)
    b.add_argument("--out", required=True)
    c = sub.add_parser("sq")
    c.add_argument("csv", nargs="+")
    args = ap.parse_args(argv)
    if args.cmd == "sq":
        print(sq_summary(args.csv))
        return 0
    if args.cmd == "stats":
        print(stats(args.csv))
    else:
        d = counters(args.fetch_csv, args.write_csv, args.n1, args.n2, args.copy_bytes)
        with open(args.out, "w") as fh:
            fh.write(json.dumps(d, indent=1) + "\n")
        print(json.dumps(d, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
