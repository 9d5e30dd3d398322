"""Summaries of rocprofv3 runs of the benchmark, for the files under profiles/.

Usage (on the results of the commands named in the summary it writes):

    python -m paper_1811_03374_amd.profsummary \
        --stats <dir>/kt/kt_kernel_stats.csv \
        --fetch <dir>/fetch/fetch_counter_collection.csv \
        --write <dir>/write/write_counter_collection.csv \
        --name <summary name> --out profiles

* ``--stats``: a ``rocprofv3 --kernel-trace --stats`` run of ``bench.py``;
  the summary lists every kernel's call count and average duration.
* ``--trace`` with ``--steps K``: the kernel trace of that run. ``bench.py``
  makes the timed steps' calls on two streams, one per depth (overlapping),
  then repeats the K steps with the calls one after another for the
  per-call figures; the summary gives the average duration per depth of
  both kinds of call: the last 2K plain dispatches are the one-after-another
  calls (depth 9, then 22), the 2K before them the overlapped ones (issued
  22, then 9).
* ``--fetch`` / ``--write``: ``rocprofv3 --pmc FETCH_SIZE`` and
  ``--pmc WRITE_SIZE`` runs of ``bench.py --traffic-probe``, which copies
  256 MiB with a plain device copy and then makes one call per depth. The
  copy calibrates the counters (bytes the counter reports for a copy of known
  size); every call's k_fused dispatch is scaled by that factor. The result is written to ``traffic.json`` together with the
  hash of the kernel source it was measured on, which ``bench.py`` checks
  before it reports the figure.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 << 20
DEPTHS = (9, 22)


def kernel_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_1811_03374_amd", "csrc", "fiberhit.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def short(name):
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0] if "(" in name else name


def read_stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append({"kernel": short(r["Name"]), "calls": int(r["Calls"]),
                    "avg_us": float(r["AverageNs"]) / 1e3, "min_us": float(r["MinNs"]) / 1e3,
                    "max_us": float(r["MaxNs"]) / 1e3, "percent": float(r["Percentage"])})
    return out


def read_counter(path, counter):
    per = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        per.setdefault(key, [short(r["Kernel_Name"]), 0.0])
        per[key][1] += float(r["Counter_Value"])
    return [(k, v[0], v[1]) for k, v in sorted(per.items())]


CALL_KERNELS = ("k_fused",)
PLAIN_KERNEL = "k_fused<0, false, false, false, true>"     # the plain single-call variant


def per_call(dispatches, factor):
    """Bytes per call, in call order (one call per depth, one k_fused
    dispatch each)."""
    return [{"k_fused": kib * 1024 * factor} for _, name, kib in dispatches if name.startswith("k_fused")]


def call_durations(trace_path, steps):
    """Average duration (us) per depth of the plain-mode calls of a bench
    run: (isolated, overlapped), each a dict depth -> us."""
    rows = [r for r in csv.DictReader(open(trace_path)) if short(r["Kernel_Name"]) == PLAIN_KERNEL]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    if len(us) < 4 * steps:
        raise SystemExit(f"{len(us)} plain dispatches in the trace, fewer than 4 x {steps}")
    iso, ovl = us[-2 * steps:], us[-4 * steps:-2 * steps]
    avg = lambda x: sum(x) / len(x)
    return ({DEPTHS[0]: avg(iso[0::2]), DEPTHS[1]: avg(iso[1::2])},
            {DEPTHS[1]: avg(ovl[0::2]), DEPTHS[0]: avg(ovl[1::2])})


def calibration(dispatches):
    for _, name, kib in dispatches:
        if "copyBuffer" in name:
            return COPY_BYTES / (kib * 1024)
    raise SystemExit("no copy dispatch found for calibration")


def sq_counters(paths):
    """Counter sums of the k_fused dispatches of ``--traffic-probe`` runs (one
    call per depth), in dispatch order, from rocprofv3 counter CSVs."""
    per = collections.OrderedDict()
    for path in paths:
        for r in csv.DictReader(open(path)):
            if "k_fused" not in r["Kernel_Name"]:
                continue
            key = (path, int(r["Dispatch_Id"]))
            per.setdefault(key, collections.Counter())[r["Counter_Name"]] += float(r["Counter_Value"])
    by_path = collections.OrderedDict()
    for (path, _), c in per.items():
        by_path.setdefault(path, []).append(c)
    out = [collections.Counter() for _ in DEPTHS]
    for calls in by_path.values():
        for j, c in enumerate(calls[:len(DEPTHS)]):
            for k, v in c.items():
                out[j].setdefault(k, v)
    return out


def sq_lines(paths, durations=None):
    cs = sq_counters(paths)
    names = sorted(set().union(*[set(c) for c in cs]))
    lines = ["| counter | " + " | ".join(f"depth {d}" for d in DEPTHS) + " |",
             "|---|" + "---|" * len(DEPTHS)]
    for n in names:
        lines.append(f"| {n} | " + " | ".join(f"{int(c.get(n, 0))}" for c in cs) + " |")
    if all("SQ_INSTS_VALU" in c for c in cs):
        issue = [c["SQ_INSTS_VALU"] / 1024 * 4 / 2.4e3 for c in cs]
        lines += ["", "VALU issue time (1024 SIMDs, 4 cycles per wave64 VALU instruction, 2.4 GHz): " +
                  ", ".join(f"depth {d}: {t:.0f} us" for d, t in zip(DEPTHS, issue)) +
                  (", against " + ", ".join(f"{u:.0f} us" for u in durations) + " per call in the kernel trace"
                   if durations else "") + "."]
    return lines


def last_call_counters(paths):
    """Counter sums of the last k_fused dispatch of each counter CSV (a probe
    whose last call is the one to read), merged over the files."""
    out = collections.Counter()
    for path in paths:
        per = collections.OrderedDict()
        for r in csv.DictReader(open(path)):
            if "k_fused" not in r["Kernel_Name"]:
                continue
            per.setdefault(int(r["Dispatch_Id"]), collections.Counter())[r["Counter_Name"]] += \
                float(r["Counter_Value"])
        if per:
            last = per[max(per)]
            for k, v in last.items():
                out.setdefault(k, v)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats")
    ap.add_argument("--sq", action="append", default=[],
                    help="rocprofv3 counter CSV of a --traffic-probe run (repeatable): SQ counter table")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--name", required=True)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--trace")
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--command", action="append", default=[],
                    help="command line that produced an input (repeatable)")
    ap.add_argument("--last-call", action="append", default=[],
                    help="rocprofv3 counter CSV whose last k_fused dispatch is summarised (repeatable)")
    ap.add_argument("--note", action="append", default=[], help="a line of text after the commands")
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    lines = [f"# {a.name}", "", "Commands:", ""]
    lines += [f"    {c}" for c in a.command] + [""]
    if a.note:
        lines += [" ".join(a.note), ""]
    if a.stats:
        stats = read_stats(a.stats)
        lines += ["| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
        for s in stats:
            lines.append(f"| {s['kernel']} | {s['calls']} | {s['avg_us']:.1f} | {s['min_us']:.1f} | "
                         f"{s['max_us']:.1f} | {s['percent']:.1f} |")
    iso = None
    if a.trace and a.steps > 0:
        iso, ovl = call_durations(a.trace, a.steps)
        lines += ["", f"Per-call durations of `{PLAIN_KERNEL}` from the kernel trace ({a.steps} steps):", "",
                  "| depth | one after another, us | overlapped (two streams), us |", "|---|---|---|"]
        for d in DEPTHS:
            lines.append(f"| {d} | {iso[d]:.1f} | {ovl[d]:.1f} |")
    if a.sq:
        lines += ["", f"SQ counters summed over the device, one `{PLAIN_KERNEL}` dispatch per depth "
                  "(`--traffic-probe`: one call at depth 9, then one at depth 22):", ""]
        lines += sq_lines(a.sq, [iso[d] for d in DEPTHS] if iso else None)
    if a.last_call:
        c = last_call_counters(a.last_call)
        lines += ["", "Counters of the last k_fused dispatch, summed over the device:", "",
                  "| counter | value |", "|---|---|"]
        lines += [f"| {k} | {int(v)} |" for k, v in sorted(c.items())]
        if "SQ_INSTS_VALU" in c:
            issue = c["SQ_INSTS_VALU"] / 1024 * 4 / 2.4e3
            lines += ["", f"VALU issue time (1024 SIMDs, 4 cycles per wave64 VALU instruction, 2.4 GHz): "
                          f"{issue:.0f} us."]
    traffic = None
    if a.fetch and a.write:
        fd = read_counter(a.fetch, "FETCH_SIZE")
        wd = read_counter(a.write, "WRITE_SIZE")
        ff, wf = calibration(fd), calibration(wd)
        fc, wc = per_call(fd, ff), per_call(wd, wf)
        traffic = {"kernel_source_sha256_16": kernel_source_hash(),
                   "calibration": {"copy_bytes": COPY_BYTES, "fetch_factor": ff, "write_factor": wf},
                   "bytes_per_launch": {}, "per_kernel": {}}
        lines += ["", "HBM traffic per call (FETCH_SIZE and WRITE_SIZE, scaled by a "
                  f"{COPY_BYTES >> 20} MiB copy: fetch x{ff:.3f}, write x{wf:.3f}):", "",
                  "| depth | kernel | fetch MB | write MB |", "|---|---|---|---|"]
        for d, f, w in zip(DEPTHS, fc, wc):
            total = sum(f.values()) + sum(w.values())
            traffic["bytes_per_launch"][str(d)] = total
            names = [k for k in CALL_KERNELS if k in f or k in w]
            traffic["per_kernel"][str(d)] = {k: {"fetch": f.get(k, 0.0), "write": w.get(k, 0.0)}
                                            for k in names}
            for k in names:
                lines.append(f"| {d} | {k} | {f.get(k, 0.0) / 1e6:.1f} | {w.get(k, 0.0) / 1e6:.1f} |")
            lines.append(f"| {d} | total | {sum(f.values()) / 1e6:.1f} | {sum(w.values()) / 1e6:.1f} |")
        with open(os.path.join(a.out, "traffic.json"), "w") as fh:
            json.dump(traffic, fh, indent=1)
    path = os.path.join(a.out, a.name + ".md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path)
    return 0


if __name__ == "__main__":
    sys.exit(main())
