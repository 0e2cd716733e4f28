"""Turn rocprofv3 output into the short text summaries kept under profiles/.

    # per-kernel durations (rocprofv3 --kernel-trace --stats)
    python -m paper_1805_04207_amd.profile_summary kstats OUT_kernel_stats.csv \\
        --cmd "<the profiled command>" --title "..." -o profiles/kernels_<workload>.md

    # per-kernel counter table from --pmc runs
    python -m paper_1805_04207_amd.profile_summary counters run1_results.db run2_results.db \\
        --cmd "<the commands>" --title "..." -o profiles/counters_<workload>.md

    # HBM traffic of one kernel from two --pmc runs (FETCH_SIZE, then WRITE_SIZE),
    # scaled by what the same counters read for the plain copy of known size
    # that `bench.py --pmc-probe` issues after the characterization
    python -m paper_1805_04207_amd.profile_summary traffic FETCH_results.db WRITE_results.db \\
        --kernel k_mem_bucket --workload "..." --copy-bytes 1073741824 \\
        --cmd "<the two commands>" -o profiles/traffic_k_mem_bucket_<workload>.md

The traffic summary ends with one machine-readable line
`traffic-json: {...}` that bench.py reads; it carries a hash of the source
files that define the kernel and of the shared headers, so that a stale
measurement is not reported for a changed kernel.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def sources_hash(kernel: str | None = None) -> str:
    """sha256 over the kernel sources and headers the library is built from;
    with `kernel`, over the headers and the source files that name it."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))):
        with open(p, "rb") as f:
            text = f.read()
        if kernel and p.endswith(".hip") and kernel.encode() not in text:
            continue
        h.update(os.path.basename(p).encode())
        h.update(text)
    return h.hexdigest()[:16]


def short_name(k: str) -> str:
    k = k.replace("(anonymous namespace)::", "")
    if k.startswith("void "):
        k = k[5:]
    return re.split(r"[<(]", k)[0]


def kstats(args) -> int:
    rows = []
    with open(args.csv) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                         float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"])))
    rows.sort(key=lambda r: -r[3])
    total = sum(r[3] for r in rows)
    out = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
           f"Kernel sources hash: `{sources_hash()}`", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for s, _, calls, tot, avg, mn, mx in rows:
        out.append(f"| {s} | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.1f} | {mn / 1e3:.1f} | "
                   f"{mx / 1e3:.1f} | {100 * tot / total:.1f} |")
    text = "\n".join(out) + "\n"
    with open(args.o, "w") as f:
        f.write(text)
    print(text)
    return 0


def _per_dispatch(db: str, counter: str):
    """{kernel short name: (mean value per dispatch, dispatches)} for one counter."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, sum(value), count(*) from counters_collection "
                       "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    acc = defaultdict(lambda: [0.0, 0])
    for k, v, n in rows:
        a = acc[short_name(k)]
        a[0] += v
        a[1] += n
    return {k: (v / n, n) for k, (v, n) in acc.items() if n}


def _largest(db: str, counter: str, kernel: str) -> float:
    """The largest per-dispatch value of a counter for one kernel (the runtime's
    copy kernel also serves many small copies; the calibration copy is the
    largest of them)."""
    con = sqlite3.connect(db)
    best = 0.0
    for k, v in con.execute("select kernel_name, value from counters_collection "
                            "where counter_name = ?", (counter,)):
        if short_name(k) == kernel:
            best = max(best, float(v))
    return best


def traffic(args) -> int:
    fetch = _per_dispatch(args.fetch_db, "FETCH_SIZE")
    write = _per_dispatch(args.write_db, "WRITE_SIZE")
    for name, d in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
        if args.kernel not in d or COPY_KERNEL not in d:
            print(f"{name}: missing {args.kernel} or {COPY_KERNEL} in {sorted(d)}", file=sys.stderr)
            return 1
    # the calibration copy reads and writes exactly copy_bytes; counters are in KiB
    cf = _largest(args.fetch_db, "FETCH_SIZE", COPY_KERNEL)
    cw = _largest(args.write_db, "WRITE_SIZE", COPY_KERNEL)
    f_scale = args.copy_bytes / (cf * 1024.0)
    w_scale = args.copy_bytes / (cw * 1024.0)
    fb = fetch[args.kernel][0] * 1024.0 * f_scale
    wb = write[args.kernel][0] * 1024.0 * w_scale
    rec = {"kernel": args.kernel, "workload": args.workload, "fetch_bytes": fb, "write_bytes": wb,
           "traffic_bytes": fb + wb, "fetch_scale": f_scale, "write_scale": w_scale,
           "sources": sources_hash(args.kernel)}
    out = [f"# HBM traffic of {args.kernel}: {args.workload}", "", "Commands:", "", "```",
           args.cmd, "```", "",
           f"Counters are KiB per dispatch, averaged over the dispatches of each kernel; the "
           f"scale factors make the plain {args.copy_bytes}-byte device copy (the largest "
           f"{COPY_KERNEL} dispatch: {cf:.0f} KiB fetched, {cw:.0f} KiB written) read and "
           f"write exactly its size.", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|---|"]
    for k in sorted(set(fetch) | set(write)):
        if k.startswith("k_") or k == COPY_KERNEL:
            fv = fetch.get(k, (float("nan"), 0))
            wv = write.get(k, (float("nan"), 0))
            out.append(f"| {k} | {max(fv[1], wv[1])} | {fv[0]:.0f} | {wv[0]:.0f} |")
    out += ["", f"Scale: fetch x{f_scale:.4f}, write x{w_scale:.4f}.  {args.kernel}: "
                f"{fb / 1e9:.3f} GB read + {wb / 1e9:.3f} GB written per launch.", "",
            "traffic-json: " + json.dumps(rec)]
    text = "\n".join(out) + "\n"
    with open(args.o, "w") as f:
        f.write(text)
    print(text)
    return 0


def counters(args) -> int:
    """Per-kernel table of the counters of one or more --pmc runs."""
    acc = defaultdict(dict)
    for db in args.dbs:
        con = sqlite3.connect(db)
        for k, c, v, n in con.execute("select kernel_name, counter_name, sum(value), count(*) "
                                      "from counters_collection group by kernel_name, "
                                      "counter_name"):
            acc[short_name(k)][c] = v / n
    names = sorted({c for d in acc.values() for c in d})
    out = [f"# {args.title}", "", "Commands:", "", "```", args.cmd, "```", "",
           f"Kernel sources hash: `{sources_hash()}`.  Values per dispatch (mean over "
           "dispatches).", "", "| kernel | " + " | ".join(names) + " |",
           "|---|" + "---|" * len(names)]
    for k in sorted(acc):
        if not k.startswith("k_"):
            continue
        out.append(f"| {k} | " + " | ".join(f"{acc[k].get(c, float('nan')):.4g}" for c in names)
                   + " |")
    text = "\n".join(out) + "\n"
    with open(args.o, "w") as f:
        f.write(text)
    print(text)
    return 0


def read_traffic(path: str, kernel: str, workload: str):
    """bench.py side: the recorded traffic in bytes per launch, or None when the
    summary is missing, for another kernel or workload, or older than the
    current kernel sources."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-json: "):
                rec = json.loads(line[len("traffic-json: "):])
                if rec.get("kernel") == kernel and rec.get("workload") == workload and \
                        rec.get("sources") == sources_hash(kernel):
                    return rec
    return None


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("kstats")
    a.add_argument("csv")
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", required=True)
    a.add_argument("-o", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_db")
    b.add_argument("write_db")
    b.add_argument("--kernel", required=True)
    b.add_argument("--workload", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--cmd", required=True)
    b.add_argument("-o", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("-o", required=True)
    args = ap.parse_args(argv)
    return {"kstats": kstats, "traffic": traffic, "counters": counters}[args.cmd_name](args)


if __name__ == "__main__":
    sys.exit(main())
