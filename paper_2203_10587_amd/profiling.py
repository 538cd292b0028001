"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2203_10587_amd.profiling stats DIR OUT.md --cmd "..."
        kernel-trace --stats run: per-kernel calls and durations.
    python -m paper_2203_10587_amd.profiling traffic --workload NAME \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-mib MIB \
        --json profiles/traffic.json --md OUT.md --cmd "..."
        FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the batched evaluation
        kernel, each scaled by what the same counter reads for a device copy of
        known size; stored under the workload name with the hash of the kernel
        sources, so bench.py reports it only while the kernel is unchanged.

Each DIR is a rocprofv3 output directory written with `-o run --output-format
csv`.  The batched evaluation kernel is the k_eval dispatch with the largest
grid; the copy kernel is the runtime's device-to-device copy (name fragment
--copy-kernel) in the calibration run.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2203_10587_amd/csrc/acopf_kernels.hip",
                  "paper_2203_10587_amd/csrc/acopf_internal.h"]


def strip_comments(src: str) -> str:
    """C/C++ source without its comments, with every run of white space
    folded to one blank (string and character literals kept as they are)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_hash() -> str:
    """Hash of the sources that define the evaluation kernel, comments and
    layout aside (so that a comment edit keeps the recorded counters)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
            h.update(b"\0")
    return h.hexdigest()[:16]


def _csv(d: str, suffix: str):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(hits[0]) as fh:
        return list(csv.DictReader(fh))


def _short(name: str) -> str:
    return name if len(name) <= 90 else name[:87] + "..."


def counter_per_dispatch(d: str, counter: str, kernel_substr: str | None):
    """{dispatch id: (grid size, kernel, value)} of one counter."""
    out = {}
    acc = defaultdict(float)
    meta = {}
    for r in _csv(d, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        if kernel_substr and kernel_substr not in r["Kernel_Name"]:
            continue
        key = int(r["Dispatch_Id"])
        acc[key] += float(r["Counter_Value"])
        meta[key] = (int(r["Grid_Size"]), r["Kernel_Name"])
    for k, v in acc.items():
        out[k] = (meta[k][0], meta[k][1], v)
    return out


def largest_grid_mean(per_dispatch: dict, skip_first: bool = True):
    """Mean counter value over the dispatches with the largest grid (the
    first such dispatch, which runs cold, is dropped when there are more)."""
    if not per_dispatch:
        raise ValueError("no dispatches")
    gmax = max(g for g, _, _ in per_dispatch.values())
    vals = [v for k, (g, _, v) in sorted(per_dispatch.items()) if g == gmax]
    if skip_first and len(vals) > 1:
        vals = vals[1:]
    name = next(n for g, n, _ in per_dispatch.values() if g == gmax)
    return sum(vals) / len(vals), len(vals), gmax, name


def _medians(d: str) -> dict:
    """Median dispatch duration (ns) per kernel name from the kernel trace
    (the average includes the first dispatches, which run before the GPU
    has reached its steady clocks)."""
    per = defaultdict(list)
    try:
        for r in _csv(d, "kernel_trace.csv"):
            per[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    except FileNotFoundError:
        return {}
    out = {}
    for k, v in per.items():
        v.sort()
        out[k] = v[len(v) // 2]
    return out


def cmd_stats(args):
    rows = _csv(args.dir, "kernel_stats.csv")
    med = _medians(args.dir)
    lines = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
             "| kernel | calls | avg us | median us | min us | max us | share |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        m = med.get(r["Name"])
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{'-' if m is None else f'{m / 1e3:.1f}'} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f}% |")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_traffic(args):
    kb = 1024.0
    fetch, nf, grid, name = largest_grid_mean(counter_per_dispatch(args.fetch, "FETCH_SIZE", "k_eval"))
    write, nw, _, _ = largest_grid_mean(counter_per_dispatch(args.write, "WRITE_SIZE", "k_eval"))
    ck = args.copy_kernel
    cf, _, _, cname = largest_grid_mean(counter_per_dispatch(args.copy_fetch, "FETCH_SIZE", ck))
    cw, _, _, _ = largest_grid_mean(counter_per_dispatch(args.copy_write, "WRITE_SIZE", ck))
    copy_bytes = args.copy_mib * (1 << 20)
    f_fetch = copy_bytes / (cf * kb)
    f_write = copy_bytes / (cw * kb)
    ent = {"kernel_hash": kernel_hash(), "kernel": name, "grid": grid,
           "fetch_kib_raw": fetch, "write_kib_raw": write,
           "copy_kernel": cname, "copy_bytes_each_way": copy_bytes,
           "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
           "fetch_scale": f_fetch, "write_scale": f_write,
           "fetch_bytes": fetch * kb * f_fetch, "write_bytes": write * kb * f_write,
           "dispatches": [nf, nw]}
    doc = {}
    if os.path.exists(args.json):
        with open(args.json) as fh:
            doc = json.load(fh)
    doc[args.workload] = ent
    with open(args.json, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    alg = f" (algorithmic {args.algorithmic / 1e6:.1f} MB)" if args.algorithmic else ""
    lines = [f"# HBM traffic of the batched evaluation kernel: {args.workload}", "",
             "Commands (each a separate rocprofv3 run):", "", "```", args.cmd, "```", "",
             f"- kernel: `{_short(name)}`, grid {grid}, mean of {nf} / {nw} warm dispatches",
             f"- FETCH_SIZE {fetch:.0f} KiB, WRITE_SIZE {write:.0f} KiB per dispatch (raw)",
             f"- copy of {copy_bytes} B each way (`{_short(cname)}`): FETCH_SIZE {cf:.0f} KiB, "
             f"WRITE_SIZE {cw:.0f} KiB -> scale {f_fetch:.3f} (fetch), {f_write:.3f} (write)",
             f"- scaled: fetch {ent['fetch_bytes'] / 1e6:.1f} MB + write {ent['write_bytes'] / 1e6:.1f} MB"
             f" = {(ent['fetch_bytes'] + ent['write_bytes']) / 1e6:.1f} MB per launch{alg}",
             f"- kernel sources hash {ent['kernel_hash']}"]
    with open(args.md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="rocprofv3 kernel trace")
    t = sub.add_parser("traffic")
    t.add_argument("--workload", required=True)
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--copy-kernel", default="copyBuffer",
                   help="name fragment of the copy kernel in the calibration run")
    t.add_argument("--algorithmic", type=float, default=0.0)
    t.add_argument("--json", required=True)
    t.add_argument("--md", required=True)
    t.add_argument("--cmd", required=True)
    args = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic}[args.what](args)


if __name__ == "__main__":
    main()
