"""Text summaries of rocprofv3 runs of the benchmark.

Two summaries are written under ``profiles/``:

* ``kernels``: the per-kernel table of a ``rocprofv3 --kernel-trace --stats``
  run (``*_kernel_stats.csv``): calls, average and total duration, share.
* ``traffic``: the HBM bytes per launch of the fused step kernel from two
  counter runs (``--pmc FETCH_SIZE`` then ``--pmc WRITE_SIZE``, KiB per
  dispatch).  Each counter is scaled by what it reads for the copy probe of
  the same run, whose bytes are known (``lb_copy_probe``: n bytes read and n
  written per dispatch).  The summary records the SHA-1 of the step-kernel
  sources, so a reader can tell whether it still describes the current kernel.

Usage::

    python -m paper_0809_4958_amd.prof_summary kernels STATS_CSV OUT --command "..." \\
        [--trace TRACE_CSV --tail N] [--tune-cache TUNE_JSONL]
    python -m paper_0809_4958_amd.prof_summary traffic FETCH_CSV WRITE_CSV OUT \\
        --copy-bytes N --command-fetch "..." --command-write "..."
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("lb_device.hpp", "lb_kernels.hpp", "lb_step.hip")


def _code_only(text: str) -> str:
    """Source text without comments, trailing blanks and blank lines, so that
    editing a comment does not count as a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash() -> str:
    """SHA-1 (16 hex digits) of the step-kernel sources' code (comments
    excluded)."""
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Readable kernel name: template arguments of the step kernels kept."""
    for k in ("k_lb", "k_chain", "k_force", "k_check", "k_finalize", "k_copy", "k_set_pre", "k_read_sites",
              "k_read_beads", "k_read"):
        if k in name:
            i = name.find(k)
            return name[i:i + 60].split("(")[0]
    # other kernels: the name without return type, namespace and argument list
    n = name.split("(")[0]
    m = re.match(r"_ZN\d+\w*?(\d+)(\w+)", n)  # an unmangled-by-the-tool C++ name: its last component
    if m and n.startswith("_ZN"):
        k = int(m.group(1))
        return m.group(2)[:k]
    n = n[5:] if n.startswith("void ") else n
    return n.split("::")[-1][:60] if "<" not in n else n[n.find("::") + 2:][:60]


def timed_average(trace_csv: str, kernel: str, tail: int):
    """Average duration (ms) of the last `tail` dispatches of `kernel` in a
    kernel-trace CSV, and how many dispatches it had in all."""
    durs = []
    for r in csv.DictReader(open(trace_csv)):
        if short_name(r.get("Kernel_Name", "")).startswith(kernel):
            durs.append((int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    durs.sort()
    last = [d for _, d in durs[-tail:]]
    return sum(last) / len(last) / 1e6, len(durs)


def kernels(stats_csv: str, out: str, command: str, trace_csv: str | None = None, tail: int = 0,
            tune_cache: str | None = None) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# rocprofv3 kernel-trace statistics", f"# command: {command}", ""]
    if tune_cache:
        lines += [f"launch shape (autotuner cache {os.path.basename(tune_cache)}):"]
        lines += ["  " + ln.strip() for ln in open(tune_cache) if ln.strip()] + [""]
    if trace_csv and tail > 0:
        avg, n = timed_average(trace_csv, "k_lb", tail)
        lines += [f"k_lb average over the last {tail} dispatches (the timed steps): {avg:.4f} ms "
                  f"({n} dispatches in all; the others are warm-up and any autotuner trials)", ""]
    lines += [f"{'kernel':48s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'share_%':>8s}"]
    for r in rows:
        name = short_name(r.get("Name", r.get("KernelName", "")))
        calls = int(float(r.get("Calls", 0)))
        avg_us = float(r.get("AverageNs", 0)) / 1e3
        tot_ms = float(r.get("TotalDurationNs", 0)) / 1e6
        pct = float(r.get("Percentage", 0))
        lines.append(f"{name:48s} {calls:7d} {avg_us:10.2f} {tot_ms:10.3f} {pct:8.2f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def per_dispatch(counter_csv: str) -> dict:
    """Mean counter value per dispatch, by (short kernel name, counter)."""
    agg = defaultdict(list)
    for r in csv.DictReader(open(counter_csv)):
        agg[(short_name(r.get("Kernel_Name", "")), r.get("Counter_Name", ""))].append(
            float(r.get("Counter_Value", 0)))
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def _pick(d: dict, kernel: str, counter: str):
    hits = [(v, n) for (k, c), (v, n) in d.items() if k.startswith(kernel) and c == counter]
    if not hits:
        raise SystemExit(f"no {counter} samples for {kernel}")
    return hits[0]


def traffic(fetch_csv: str, write_csv: str, out: str, copy_bytes: int, cmd_fetch: str,
            cmd_write: str, workload: str, storage: str, algorithmic: float) -> None:
    fd, wd = per_dispatch(fetch_csv), per_dispatch(write_csv)
    cf, ncf = _pick(fd, "k_copy", "FETCH_SIZE")
    cw, ncw = _pick(wd, "k_copy", "WRITE_SIZE")
    lf, nlf = _pick(fd, "k_lb", "FETCH_SIZE")
    lw, nlw = _pick(wd, "k_lb", "WRITE_SIZE")
    kf = copy_bytes / (cf * 1024.0)
    kw = copy_bytes / (cw * 1024.0)
    fetch_b = lf * 1024.0 * kf
    write_b = lw * 1024.0 * kw
    lines = [
        "# HBM traffic of the fused step kernel k_lb from two rocprofv3 counter runs",
        f"# command (FETCH_SIZE): {cmd_fetch}",
        f"# command (WRITE_SIZE): {cmd_write}",
        "# counters are KiB per dispatch; each is scaled by its reading for the copy probe",
        "# (k_copy: copy_bytes read and copy_bytes written per dispatch)",
        f"workload: {workload}",
        f"storage: {storage}",
        f"kernel_sources_sha1: {kernel_source_hash()}",
        f"copy_bytes: {copy_bytes}",
        f"copy_fetch_kib_per_dispatch: {cf:.6g} ({ncf} dispatches)",
        f"copy_write_kib_per_dispatch: {cw:.6g} ({ncw} dispatches)",
        f"fetch_scale: {kf:.4f}",
        f"write_scale: {kw:.4f}",
        f"k_lb_fetch_kib_per_dispatch: {lf:.6g} ({nlf} dispatches)",
        f"k_lb_write_kib_per_dispatch: {lw:.6g} ({nlw} dispatches)",
        f"hbm_read_bytes_per_launch: {fetch_b:.6g}",
        f"hbm_write_bytes_per_launch: {write_b:.6g}",
        f"hbm_bytes_per_launch: {fetch_b + write_b:.6g}",
        f"algorithmic_bytes_per_launch: {algorithmic:.6g}",
        f"traffic_over_algorithmic: {(fetch_b + write_b) / algorithmic:.4f}",
    ]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("stats_csv")
    k.add_argument("out")
    k.add_argument("--command", required=True)
    k.add_argument("--trace", help="kernel_trace.csv of the same run")
    k.add_argument("--tail", type=int, default=0, help="timed k_lb dispatches at the end of the run")
    k.add_argument("--tune-cache", help="autotuner cache the profiled run used")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("out")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--storage", required=True)
    t.add_argument("--algorithmic", type=float, required=True,
                   help="algorithmic bytes per k_lb launch (bench.py roofline)")
    a = p.parse_args()
    if a.what == "kernels":
        kernels(a.stats_csv, a.out, a.command, a.trace, a.tail, a.tune_cache)
    else:
        traffic(a.fetch_csv, a.write_csv, a.out, a.copy_bytes, a.command_fetch, a.command_write,
                a.workload, a.storage, a.algorithmic)


if __name__ == "__main__":
    main()
