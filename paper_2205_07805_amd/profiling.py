"""Summaries of rocprofv3 output for the solver's kernels.

Two inputs, both CSV files written by rocprofv3 for a run of ``bench.py``:

* a kernel trace (``--kernel-trace --stats``): per-kernel launch counts and
  average durations over the launches that did work, per family (operator
  apply, fused reduction, basis update, ...), with the iteration index j of
  each launch recovered from the dispatch order;
* two counter runs (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, KiB per
  dispatch): HBM bytes per launch, each counter scaled by what it reads for a
  plain device copy of known size (``bench.py --copy-calibration``), next to
  the algorithmic bytes of the same launches.

Usage::

    python -m paper_2205_07805_amd.profiling trace TRACE.csv [--solves a:b]
    python -m paper_2205_07805_amd.profiling traffic FETCH.csv WRITE.csv \
        --n N --nnz NNZ --workload NAME [--out FILE.json]

Nothing here touches the GPU.
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
KERNEL_SRC = os.path.join(HERE, "csrc", "kernels.hip")

# launches that return at once (a cycle ended before them) take about a
# microsecond; any launch that streams data takes several
NOOP_US = 4.0


def code_sha(text: str) -> str:
    """Hash of C++ source with comments and whitespace removed: edits to
    comments do not change it, edits to code do."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = re.sub(r"\s+", " ", text).strip()
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def kernel_source_sha() -> str:
    with open(KERNEL_SRC, encoding="utf-8") as f:
        return code_sha(f.read())


def short_name(name: str) -> str:
    s = re.sub(r"^void ", "", name)
    return s.split("(")[0]


def family(name: str) -> str | None:
    s = short_name(name)
    if not s.startswith("igs::"):
        return None
    for key in ("spmv_csr_kernel", "spmv_ell_kernel", "gemv_dense_kernel", "gemv_mfma_kernel"):
        if key in s:
            return "spmv"
    # (a name can hold another's: opreduce_kernel holds reduce_kernel and
    # xupdate_kernel holds update_kernel, so the longer names come first)
    for key, fam in (("opreduce_kernel", "opreduce"), ("reduce_kernel", "reduce"),
                     ("xupdate_kernel", "xupdate"), ("update_kernel", "update"),
                     ("coef_kernel", "coef"), ("lsq_kernel", "lsq"),
                     ("cycle_begin_kernel", "cycle_begin"), ("bnorm_kernel", "bnorm")):
        if key in s:
            return fam
    return s


def _rows(path):
    with open(path) as f:
        rows = list(csv.DictReader(f))
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    rows.sort(key=lambda r: int(r[key]))
    return rows


def label_launches(rows):
    """Tag every solver launch with (solve, family, j, cycle).  A solve starts
    at bnorm_kernel, a cycle at cycle_begin_kernel; the operator apply right
    after cycle_begin is the explicit residual, later ones belong to
    iteration j of the cycle (reduce launches count j)."""
    out = []
    solve = -1
    cycle = -1
    j = -1
    after_begin = False
    for r in rows:
        fam = family(r["Kernel_Name"])
        if fam is None:
            out.append(None)
            continue
        if fam == "bnorm":
            solve += 1
        if fam == "cycle_begin":
            j = -1
            cycle += 1
            after_begin = True
            out.append((solve, fam, None, cycle))
            continue
        if fam == "spmv":
            if after_begin:
                out.append((solve, "residual", None, cycle))
                after_begin = False
                continue
            out.append((solve, "spmv", j + 1, cycle))
            continue
        if fam in ("reduce", "opreduce"):
            j += 1
            out.append((solve, fam, j, cycle))
            continue
        out.append((solve, fam, j if fam in ("update", "coef") else None, cycle))
    return out


def trace_summary(trace_csv: str, solves=None) -> str:
    rows = _rows(trace_csv)
    labels = label_launches(rows)
    nsolves = 1 + max((l[0] for l in labels if l), default=-1)
    lo, hi = solves if solves else (0, nsolves)
    per = collections.defaultdict(list)
    perj = collections.defaultdict(list)
    noop = collections.Counter()
    # a reduction that returned at once marks its iteration as not run; the
    # operator apply of that iteration was gated off too
    idle = set()
    for r, l in zip(rows, labels):
        if l and l[1] in ("reduce", "opreduce") and \
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 < NOOP_US:
            idle.add((l[3], l[2]))
    for r, l in zip(rows, labels):
        if l is None or not (lo <= l[0] < hi):
            continue
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if (l[1] in ("reduce", "opreduce", "update", "coef") and us < NOOP_US) or \
                (l[1] == "spmv" and (l[3], l[2]) in idle):
            noop[l[1]] += 1
            continue
        per[l[1]].append(us)
        if l[2] is not None:
            perj[(l[1], l[2])].append(us)
    lines = [f"solves {lo}..{hi - 1} of {nsolves} in the trace (a solve starts at bnorm_kernel)",
             f"launches queued after their cycle ended (returned at once) excluded: "
             + ", ".join(f"{k} {v}" for k, v in sorted(noop.items())),
             "", f"{'family':12s} {'launches':>8s} {'avg_us':>9s} {'total_ms':>9s}"]
    tot = sum(sum(v) for v in per.values())
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k:12s} {len(v):8d} {sum(v) / len(v):9.2f} {sum(v) / 1e3:9.2f}"
                     f"  ({100 * sum(v) / tot:4.1f}%)")
    lines += ["", "per iteration j (average us): opreduce  reduce  update  spmv  coef"]
    js = sorted({j for (_, j) in perj})
    for j in js:
        if j % 5 and j != js[-1]:
            continue
        f = lambda k: (sum(perj[(k, j)]) / len(perj[(k, j)])) if perj.get((k, j)) else float("nan")
        lines.append(f"  j={j:3d} {f('opreduce'):8.2f} {f('reduce'):8.2f} {f('update'):8.2f} "
                     f"{f('spmv'):8.2f} {f('coef'):8.2f}")
    return "\n".join(lines)


def _calibration(rows):
    """KiB the counter reads for the plain device copies that bench.py
    --copy-calibration runs before any solver kernel: the 256 MiB copy (the
    largest reading) and the 64 MiB one (the smallest of the large ones, a
    cross-check of the scale), or None for the second when absent."""
    vals = []
    for r in rows:
        if short_name(r["Kernel_Name"]).startswith("igs::"):
            break
        if "copyBuffer" in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit("no calibration copy before the first solver kernel "
                         "(run bench.py with --copy-calibration)")
    big = max(vals)
    # the 64 MiB copy reads about a quarter of the 256 MiB one
    small = [v for v in vals if 0.15 * big < v < 0.4 * big]
    return big, (max(small) if small else None)


def algorithmic_bytes(fam, j, n, nnz, m):
    if fam == "opreduce":
        # the operator's arrays, z written once, V_{0:j} and u read once
        return 12.0 * nnz + 4.0 * (n + 1) + 8.0 * n + 8.0 * n * (j + 1)
    if fam == "reduce":
        return 8.0 * n * (j + 1) + (8.0 * n if j < m else 0.0)
    if fam == "update":
        return 8.0 * n * (j + 1) + 24.0 * n
    if fam == "spmv":
        return 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n
    return None


def traffic(fetch_csv, write_csv, n, nnz, m, workload, solve=0, copy_bytes=256 * 2**20):
    f_rows, w_rows = _rows(fetch_csv), _rows(write_csv)
    (cf, cf64), (cw, cw64) = _calibration(f_rows), _calibration(w_rows)
    sf, sw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    # pair fetch and write launches by order within (family, j)
    fam_launch = collections.defaultdict(list)
    for rows, key in ((f_rows, "fetch"), (w_rows, "write")):
        seq = collections.defaultdict(list)
        for r, l in zip(rows, label_launches(rows)):
            if l is None or l[0] != solve or l[1] not in ("spmv", "opreduce", "reduce", "update"):
                continue
            seq[(l[1], l[2])].append(float(r["Counter_Value"]) * 1024.0 * (sf if key == "fetch" else sw))
        fam_launch[key] = seq
    out = {"kernel_source_sha": kernel_source_sha(), "workload": workload,
           "calibration": {"copy_bytes_read_and_written": copy_bytes,
                           "FETCH_SIZE_KiB": cf, "WRITE_SIZE_KiB": cw,
                           "fetch_scale": sf, "write_scale": sw,
                           # the same scale from the 64 MiB copy
                           "fetch_scale_64MiB": (copy_bytes / 4) / (cf64 * 1024.0) if cf64 else None,
                           "write_scale_64MiB": (copy_bytes / 4) / (cw64 * 1024.0) if cw64 else None},
           "kernels": {}}
    for fam in ("spmv", "opreduce", "reduce", "update"):
        fetch = write = alg = 0.0
        cnt = 0
        for (fm, j), fv in fam_launch["fetch"].items():
            if fm != fam:
                continue
            wv = fam_launch["write"].get((fm, j), [])
            for k, fb in enumerate(fv):
                a = algorithmic_bytes(fm, j, n, nnz, m)
                if fb < 0.01 * a:  # queued after the cycle ended: returned at once
                    continue
                fetch += fb
                write += wv[k] if k < len(wv) else 0.0
                alg += a
                cnt += 1
        if cnt:
            out["kernels"][fam] = {"launches": cnt,
                                   "hbm_bytes_per_launch": (fetch + write) / cnt,
                                   "fetch_bytes_per_launch": fetch / cnt,
                                   "write_bytes_per_launch": write / cnt,
                                   "algorithmic_bytes_per_launch": alg / cnt,
                                   "hbm_over_algorithmic": (fetch + write) / alg}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--solves", default=None, help="a:b, the solves (0-based) to summarise")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--n", type=int, required=True)
    c.add_argument("--nnz", type=int, required=True)
    c.add_argument("--restart", type=int, required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--solve", type=int, default=0)
    c.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        sl = tuple(int(x) for x in a.solves.split(":")) if a.solves else None
        print(trace_summary(a.csv, sl))
    else:
        res = traffic(a.fetch_csv, a.write_csv, a.n, a.nnz, a.restart, a.workload, a.solve)
        txt = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(txt + "\n")
        print(txt)


if __name__ == "__main__":
    sys.exit(main())
