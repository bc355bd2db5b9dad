"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_1602_08604_amd.profsum stats   --dir D --out F.txt --command CMD [--kernel REGEX]
    python -m paper_1602_08604_amd.profsum counters --dirs D... --commands CMD... --kernel REGEX --out F.txt
    python -m paper_1602_08604_amd.profsum traffic --fetch-dir D1 --write-dir D2 \
        --kernel REGEX [--sum-kernels] --copy-kernel REGEX --copy-bytes B --out-json F.json --out-txt F.txt \
        --command-fetch CMD1 --command-write CMD2

`stats` turns a `rocprofv3 --kernel-trace --stats` kernel_stats CSV into a short text
table.  `traffic` turns two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs into
HBM bytes per launch of the selected kernel, each counter scaled by what it reads for
a plain copy kernel of known size run in the same program (FETCH_SIZE counts in KiB
and, on this device, reports about half of the bytes a streaming read moves).
The JSON record carries a hash of the kernel sources so that a reader can tell
whether it still describes the current kernels.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_1602_08604_amd/csrc/lre_kernels.hpp", "paper_1602_08604_amd/csrc/lre_abi.hip")
BATCH_SOURCES = KERNEL_SOURCES + ("paper_1602_08604_amd/csrc/lre_batch.hip",)


def kernel_source_hash(workload: str = "") -> str:
    """Hash of the sources the workload's kernels are built from (the batch kernel also
    lives in lre_batch.hip)."""
    h = hashlib.sha256()
    for rel in (BATCH_SOURCES if workload == "batch" else KERNEL_SOURCES):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)
    name = re.sub(r"^void ", "", name)
    name = re.sub(r"lre::|at::native::", "", name)
    return name


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def stats(args):
    rows = list(csv.DictReader(open(_find(args.dir, "kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    if args.kernel:
        rows = [r for r in rows if re.search(args.kernel, short_name(r["Name"]))]
    lines = [f"# rocprofv3 kernel statistics", "", f"command: {args.command}", "",
             f"{'kernel':72s} {'calls':>6s} {'avg_ms':>10s} {'min_ms':>10s} {'max_ms':>10s} {'pct':>6s}"]
    for r in rows[: args.top]:
        lines.append(f"{short_name(r['Name'])[:72]:72s} {int(r['Calls']):6d} "
                     f"{float(r['AverageNs']) / 1e6:10.4f} {float(r['MinNs']) / 1e6:10.4f} "
                     f"{float(r['MaxNs']) / 1e6:10.4f} {float(r['Percentage']):6.2f}")
    if args.note:
        lines += ["", args.note]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_means(d: str, counter: str):
    """Mean counter value per dispatch for each kernel name."""
    per = {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        key = (short_name(r["Kernel_Name"]), r.get("Dispatch_Id", ""))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (k, _), v in per.items():
        out.setdefault(k, []).append(v)
    return {k: (statistics.mean(v), len(v)) for k, v in out.items()}


def _pick(means, regex):
    hits = [(k, v) for k, v in means.items() if re.search(regex, k)]
    if not hits:
        raise SystemExit(f"no kernel matches {regex!r}; have {sorted(means)}")
    hits.sort(key=lambda kv: -kv[1][1])
    return hits[0]


def _sum_all(means, regex):
    """Every kernel matching regex, summed per dispatch (kernels launched once each per
    step of a multi-kernel launch)."""
    hits = sorted((k, v) for k, v in means.items() if re.search(regex, k))
    if not hits:
        raise SystemExit(f"no kernel matches {regex!r}; have {sorted(means)}")
    return " + ".join(k for k, _ in hits), (sum(v[0] for _, v in hits), min(v[1] for _, v in hits))


def traffic(args):
    fetch = _counter_means(args.fetch_dir, "FETCH_SIZE")
    write = _counter_means(args.write_dir, "WRITE_SIZE")
    pick = _sum_all if args.sum_kernels else _pick
    kname, (f_kib, f_n) = pick(fetch, args.kernel)
    _, (w_kib, w_n) = pick(write, args.kernel)
    cname, (cf_kib, _) = _pick(fetch, args.copy_kernel)
    _, (cw_kib, _) = _pick(write, args.copy_kernel)
    f_read = args.copy_bytes / (cf_kib * 1024.0)
    f_write = args.copy_bytes / (cw_kib * 1024.0)
    read_b = f_kib * 1024.0 * f_read
    write_b = w_kib * 1024.0 * f_write
    rec = {
        "kernel": kname,
        "workload": args.workload,
        "kernel_source_hash": kernel_source_hash(args.workload),
        "hbm_bytes_per_launch": read_b + write_b,
        "read_bytes_per_launch": read_b,
        "write_bytes_per_launch": write_b,
        "fetch_size_kib": f_kib, "write_size_kib": w_kib, "dispatches": [f_n, w_n],
        "copy_kernel": cname, "copy_bytes_each_way": args.copy_bytes,
        "copy_fetch_size_kib": cf_kib, "copy_write_size_kib": cw_kib,
        "scale_read": f_read, "scale_write": f_write,
        "command_fetch": args.command_fetch, "command_write": args.command_write,
    }
    with open(args.out_json, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# HBM traffic of {kname} ({args.workload})", "",
             f"fetch run: {args.command_fetch}", f"write run: {args.command_write}", "",
             f"FETCH_SIZE {f_kib:.6g} KiB/dispatch (x{f_n}), WRITE_SIZE {w_kib:.6g} KiB/dispatch (x{w_n})",
             f"copy kernel {cname}: {args.copy_bytes} B each way -> FETCH_SIZE {cf_kib:.6g} KiB, "
             f"WRITE_SIZE {cw_kib:.6g} KiB; scale read {f_read:.4f}, write {f_write:.4f}",
             f"HBM bytes per launch: read {read_b / 1e9:.4f} GB + write {write_b / 1e9:.4f} GB "
             f"= {(read_b + write_b) / 1e9:.4f} GB",
             f"kernel source hash {rec['kernel_source_hash']}"]
    with open(args.out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(args):
    """Mean per dispatch of every counter in the runs, for the kernels matching --kernel."""
    lines = [f"# rocprofv3 counters of kernels matching {args.kernel!r}", ""]
    for d, cmd in zip(args.dirs, args.commands):
        lines.append(f"run: {cmd}")
        per = {}
        for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
            name = short_name(r["Kernel_Name"])
            if not re.search(args.kernel, name):
                continue
            key = (name, r["Counter_Name"], r.get("Dispatch_Id", ""))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        agg = {}
        for (name, ctr, _), v in per.items():
            agg.setdefault((name, ctr), []).append(v)
        for (name, ctr), v in sorted(agg.items()):
            lines.append(f"  {name[:60]:60s} {ctr:28s} {statistics.mean(v):16.6g} (x{len(v)})")
        lines.append("")
    if args.note:
        lines.append(args.note)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--dirs", nargs="+", required=True)
    c.add_argument("--commands", nargs="+", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--note", default="")
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--top", type=int, default=14)
    s.add_argument("--kernel", default="", help="keep only kernels matching this regex")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch-dir", required=True)
    t.add_argument("--write-dir", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--sum-kernels", action="store_true",
                   help="sum every kernel matching --kernel (one launch made of several kernels)")
    t.add_argument("--copy-kernel", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out-json", required=True)
    t.add_argument("--out-txt", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    main()
