"""Summaries of rocprofv3 output for the solver's kernels.

    python -m paper_1801_08655_amd.rocprof_summary stats <dir> [--match REGEX]
    python -m paper_1801_08655_amd.rocprof_summary traffic <fetch_dir> <write_dir>
        --kernel REGEX --copy REGEX --copy-bytes N --class NAME --out FILE
    python -m paper_1801_08655_amd.rocprof_summary mfma <dir> --class LABEL=REGEX ...
    python -m paper_1801_08655_amd.rocprof_summary timeline <dir> --class LABEL=REGEX ...
        [--flops-from PMC_DIR]

``stats`` prints the per-kernel table of a ``--kernel-trace --stats`` run.
``traffic`` combines a ``--pmc FETCH_SIZE`` run and a ``--pmc WRITE_SIZE``
run: the counters of a plain device copy of known size calibrate the
counters (bytes per counted KiB), and the kernels matching ``--kernel`` get
their HBM bytes per dispatch from the calibrated counters.  The result is
written as ``key: value`` lines, with a hash of the substitution kernel
sources so that a later run can tell whether the figures still describe
the code.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/kernels_solve.hip", "csrc/kernels_common.h", "csrc/kernels.h"]


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits


def read_stats(d):
    rows = []
    for path in _find(d, "*kernel_stats.csv"):
        with open(path) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def read_counters(d, counter):
    """[(kernel name, value)] of every dispatch for one counter, in dispatch
    order (values of one dispatch summed over its records)."""
    acc = {}
    for path in _find(d, "*counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    key = int(r.get("Dispatch_Id", 0) or 0)
                    name, v = acc.get(key, (r["Kernel_Name"], 0.0))
                    acc[key] = (name, v + float(r["Counter_Value"]))
    return [acc[k] for k in sorted(acc)]


def read_trace(d):
    """[(kernel name, duration ns)] of every dispatch, in dispatch order."""
    rows = []
    for path in _find(d, "*kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r.get("Dispatch_Id", 0) or 0), r["Kernel_Name"],
                             int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    return [(n, t) for _, n, t in rows]


def _short(name):
    """A kernel name without its namespace prefix and argument list."""
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("helm::kern::(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return n[:i]
    return n[:90]


def cmd_stats(a):
    if a.last:
        # the last N dispatches of the matching kernels: the timed steps of a
        # run whose earlier dispatches were warm-up and one-time set-up
        rx = re.compile(a.match)
        sel = [t for n, t in read_trace(a.dir) if rx.search(n)][-a.last:]
        print(f"last {len(sel)} dispatches matching `{a.match}`: "
              f"average {sum(sel) / len(sel) / 1e3:.2f} us, total {sum(sel) / 1e6:.3f} ms")
        return
    rows = read_stats(a.dir)
    rx = re.compile(a.match) if a.match else None
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        if rx and not rx.search(r["Name"]):
            continue
        print(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")


def cmd_traffic(a):
    kx, cx = re.compile(a.kernel), re.compile(a.copy)
    res = {"kernel_class": a.cls, "kernel_regex": a.kernel,
           "sources_sha256": kernel_sources_hash(), "copy_bytes": a.copy_bytes}
    for counter, d in (("FETCH_SIZE", a.fetch_dir), ("WRITE_SIZE", a.write_dir)):
        vals = read_counters(d, counter)
        ker = [v for n, v in vals if kx.search(n)]
        if a.last:
            ker = ker[-a.last:]
        cop = [v for n, v in vals if cx.search(n) and not kx.search(n)]
        if not ker or not cop:
            raise SystemExit(f"{counter}: {len(ker)} kernel and {len(cop)} copy dispatches")
        copy_kib = max(cop)                      # the calibration copy is the largest
        scale = a.copy_bytes / copy_kib          # bytes per counted KiB
        key = counter.lower()
        res[f"{key}_dispatches"] = len(ker)
        res[f"{key}_kib_per_dispatch"] = sum(ker) / len(ker)
        res[f"{key}_copy_kib"] = copy_kib
        res[f"{key}_bytes_per_kib"] = scale
        res[f"{key}_bytes_per_dispatch"] = sum(ker) / len(ker) * scale
    res["hbm_bytes_per_launch"] = res["fetch_size_bytes_per_dispatch"] + \
        res["write_size_bytes_per_dispatch"]
    with open(a.out, "w") as fh:
        for k, v in res.items():
            fh.write(f"{k}: {v}\n")
        if a.note:
            fh.write(f"note: {a.note}\n")
    print(open(a.out).read())


def cmd_mfma(a):
    """Matrix-core counters of the dispatches matching each class regex: the
    executed MFMA flops (SQ_INSTS_VALU_MFMA_MOPS_F32 x 512, or _F64) and the
    busy fraction of the matrix cores, SQ_VALU_MFMA_BUSY_CYCLES (summed over
    the SIMDs) over SIMDs x the active cycles of one XCD (GRBM_GUI_ACTIVE is
    summed over the XCDs), over the last N dispatches."""
    acc = {}
    for path in _find(a.dir, "*counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                key = int(r.get("Dispatch_Id", 0) or 0)
                d = acc.setdefault(key, {"name": r["Kernel_Name"],
                                         "t": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
                d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    disp = [acc[k] for k in sorted(acc)]
    print("| class | dispatches | executed MFMA GFLOP / dispatch | MFMA busy | executed TFLOP/s |")
    print("|---|---|---|---|---|")
    for spec in a.cls:
        label, rx = spec.split("=", 1)
        sel = [d for d in disp if re.search(rx, d["name"])]
        if a.last:
            sel = sel[-a.last:]
        if not sel:
            continue
        mops = sum(d.get(f"SQ_INSTS_VALU_MFMA_MOPS_{a.dtype}", 0.0) for d in sel)
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in sel)
        active = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in sel)
        t = sum(d["t"] for d in sel)
        flops = 512.0 * mops
        util = busy / (active / a.xcds * a.simds) if active else float("nan")
        print(f"| {label} | {len(sel)} | {flops / len(sel) / 1e9:.2f} | {util:.3f} | "
              f"{flops / t / 1e3:.1f} |")


def read_intervals(d):
    """[(start ns, end ns, kernel name, queue)] of every dispatch of a
    ``--kernel-trace`` run, sorted by start."""
    rows = []
    for path in _find(d, "*kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                q = r.get("Stream_Id") or r.get("Queue_Id") or "0"
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                             r["Kernel_Name"], q))
    rows.sort()
    return rows


def _union(iv):
    """Total length covered by the intervals [(start, end)] (sorted by start)."""
    tot, cur_s, cur_e = 0, None, None
    for s, e in iv:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot


def cmd_timeline(a):
    """Concurrency of a kernel trace: the span from the first start to the
    last end, the time at least one kernel runs, the mean number of kernels
    in flight while any runs (summed durations over covered time), the
    distinct streams, and per class the summed kernel time, the time the
    class covers and, with --flops-from (a ``--pmc`` run of the same command
    with SQ_INSTS_VALU_MFMA_MOPS_F32), the executed MFMA flops over the time
    the class covers."""
    rows = read_intervals(a.dir)
    if a.window_match:
        # the dispatches from the start of the window_from-th last match to the
        # start of the window_to-th last match (0: to the end of the trace)
        rx = re.compile(a.window_match)
        starts = [s for s, _, n, _ in rows if rx.search(n)]
        lo = starts[-a.window_from]
        hi = starts[-a.window_to] if a.window_to > 0 else float("inf")
        rows = [r for r in rows if lo <= r[0] < hi]
        print(f"window: from the {a.window_from}-th last to the "
              f"{a.window_to or 'end'}-th last dispatch matching `{a.window_match}`")
    if not rows:
        raise SystemExit("empty trace")
    span = max(e for _, e, _, _ in rows) - rows[0][0]
    busy = _union([(s, e) for s, e, _, _ in rows])
    summed = sum(e - s for s, e, _, _ in rows)
    # peak number of kernels in flight
    ev = sorted([(s, 1) for s, _, _, _ in rows] + [(e, -1) for _, e, _, _ in rows])
    cur = peak = 0
    for _, d in ev:
        cur += d
        peak = max(peak, cur)
    print(f"dispatches: {len(rows)}; streams: {len({q for *_, q in rows})}")
    print(f"span {span / 1e9:.3f} s; some kernel running {busy / 1e9:.3f} s "
          f"({busy / span:.3f} of the span); summed kernel time {summed / 1e9:.3f} s; "
          f"mean kernels in flight while busy {summed / busy:.2f}; peak {peak}")
    mops = {}
    if a.flops_from:
        for spec in a.cls:
            label, rx = spec.split("=", 1)
            vals = read_counters(a.flops_from, "SQ_INSTS_VALU_MFMA_MOPS_F32")
            mops[label] = sum(v for n, v in vals if re.search(rx, n))
    print("| class | dispatches | summed ms | covered ms | mean in flight | executed TFLOP/s over covered time |")
    print("|---|---|---|---|---|---|")
    for spec in a.cls:
        label, rx = spec.split("=", 1)
        sel = [(s, e) for s, e, n, _ in rows if re.search(rx, n)]
        if not sel:
            continue
        cov = _union(sel)
        tot = sum(e - s for s, e in sel)
        rate = f"{512.0 * mops[label] / cov / 1e3:.1f}" if label in mops else "-"
        print(f"| {label} | {len(sel)} | {tot / 1e6:.1f} | {cov / 1e6:.1f} | {tot / cov:.2f} | {rate} |")
    if a.top > 0:
        # the kernels with the most summed time in the trace (or window)
        per = {}
        for s0, e0, n, _ in rows:
            c, t = per.get(n, (0, 0))
            per[n] = (c + 1, t + e0 - s0)
        print()
        print("| kernel | dispatches | summed ms | share of the summed time |")
        print("|---|---|---|---|")
        for n, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1])[:a.top]:
            print(f"| `{_short(n)}` | {c} | {t / 1e6:.1f} | {t / summed:.3f} |")


def read_traffic(path):
    """Parsed ``key: value`` file written by ``traffic`` (None if missing)."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as fh:
        for line in fh:
            if ": " in line:
                k, v = line.rstrip("\n").split(": ", 1)
                try:
                    out[k] = float(v)
                except ValueError:
                    out[k] = v
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--match", default=None)
    s.add_argument("--last", type=int, default=0)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--class", dest="cls", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--note", default="")
    t.add_argument("--last", type=int, default=0)
    m = sub.add_parser("mfma")
    m.add_argument("dir")
    m.add_argument("--class", dest="cls", action="append", required=True,
                   help="LABEL=REGEX of a kernel class (repeatable)")
    m.add_argument("--last", type=int, default=0)
    m.add_argument("--dtype", default="F32")
    m.add_argument("--simds", type=int, default=1024)
    m.add_argument("--xcds", type=int, default=8)
    tl = sub.add_parser("timeline")
    tl.add_argument("dir")
    tl.add_argument("--class", dest="cls", action="append", default=[],
                    help="LABEL=REGEX of a kernel class (repeatable)")
    tl.add_argument("--flops-from", default=None,
                    help="directory of a --pmc SQ_INSTS_VALU_MFMA_MOPS_F32 run of the same command")
    tl.add_argument("--window-match", default=None,
                    help="restrict to a window delimited by dispatches matching this regex")
    tl.add_argument("--window-from", type=int, default=0)
    tl.add_argument("--window-to", type=int, default=0)
    tl.add_argument("--top", type=int, default=0,
                    help="also list the N kernels with the most summed time")
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "mfma": cmd_mfma,
     "timeline": cmd_timeline}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
