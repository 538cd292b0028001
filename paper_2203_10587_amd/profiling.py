"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2203_10587_amd.profiling stats DIR OUT.md --cmd "..." [--by-grid]
        kernel-trace --stats run: per-kernel calls and durations (per kernel
        and launch size with --by-grid).
    python -m paper_2203_10587_amd.profiling counters DIR [DIR ...] --out OUT.md --cmd "..."
        occupancy, stall and L2 counters per kernel (one DIR per counter set).
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


def _by_grid(d: str):
    """Per (kernel, grid size) from the kernel trace: calls, mean, median,
    min, max in ns (one kernel template can serve launches of different
    sizes: a schedule's persistent grid, another formulation's batch)."""
    per = defaultdict(list)
    for r in _csv(d, "kernel_trace.csv"):
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        per[(r["Kernel_Name"], g)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = []
    for (name, g), v in per.items():
        v.sort()
        out.append((name, g, len(v), sum(v) / len(v), v[len(v) // 2], v[0], v[-1]))
    out.sort(key=lambda t: -t[2] * t[3])
    return out


def cmd_stats(args):
    if args.by_grid:
        lines = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
                 "Per kernel and launch size (workgroups x threads), from the kernel trace:", "",
                 "| kernel | grid | calls | avg us | median us | min us | max us |",
                 "|---|---|---|---|---|---|---|"]
        for name, g, n, avg, med, mn, mx in _by_grid(args.dir):
            if args.kernel and args.kernel not in name:
                continue
            lines.append(f"| `{_short(name)}` | {g} | {n} | {avg / 1e3:.1f} | {med / 1e3:.1f} | "
                         f"{mn / 1e3:.1f} | {mx / 1e3:.1f} |")
        with open(args.out, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
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


XCDS = 8  # GRBM_GUI_ACTIVE comes summed over the accelerator complex dies


def _counter_table(dirs):
    """{(kernel, grid): {counter: mean per dispatch}} over the given pmc runs;
    per kernel only the grid size seen most often (the batched launch), the
    first of its dispatches dropped when there are more."""
    acc = defaultdict(lambda: defaultdict(float))
    meta = {}
    for d in dirs:
        for r in _csv(d, "counter_collection.csv"):
            key = (d, int(r["Dispatch_Id"]))
            acc[key][r["Counter_Name"]] += float(r["Counter_Value"])
            meta[key] = (r["Kernel_Name"], int(r["Grid_Size"]), int(r["VGPR_Count"]),
                         int(r["LDS_Block_Size"]),
                         int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    by = defaultdict(list)
    for key, cnt in acc.items():
        by[(key[0], meta[key][0], meta[key][1])].append((key[1], cnt, meta[key]))
    best = {}
    for (d, name, grid), lst in by.items():
        k = (name, grid)
        cur = best.setdefault(k, {"n": 0, "vals": defaultdict(list), "meta": lst[0][2]})
        lst.sort()
        if len(lst) > 1:
            lst = lst[1:]
        for _, cnt, m in lst:
            for c, v in cnt.items():
                cur["vals"][c].append(v)
        cur["n"] = max(cur["n"], len(lst))
        cur.setdefault("dur", []).extend(m[4] for _, _, m in lst)
    # keep the modal grid of each kernel
    out = {}
    for (name, grid), ent in best.items():
        prev = out.get(name)
        if prev is None or ent["n"] > prev[1]["n"]:
            out[name] = (grid, ent)
    return out


def cmd_counters(args):
    tab = _counter_table(args.dirs)
    lines = [f"# {args.title}", "", "Commands (one rocprofv3 run per counter set):", "", "```",
             args.cmd, "```", "",
             "Per dispatch of each kernel's batched launch (mean over its warm dispatches). "
             "Derived: waves/CU = 4 SQ_WAVE_CYCLES / (active cycles x CUs) with "
             f"active cycles = GRBM_GUI_ACTIVE / {XCDS} (the counter is summed over the dies) "
             "and SQ_WAVE_CYCLES in quad-cycles; wait, issue-wait and active are SQ_WAIT_ANY, "
             "SQ_WAIT_INST_ANY and SQ_ACTIVE_INST_ANY as fractions of SQ_WAVE_CYCLES; L2 hit = "
             "TCC_HIT / TCC_REQ; HBM reads = TCC_EA0_RDREQ; L1->L2 = TCP_TCC_READ_REQ and "
             "TCP_TCC_WRITE_REQ; per instance = divided by --instances.", "",
             "| kernel | grid | VGPR | LDS B | us | waves/CU | wait | issue-wait | active | "
             "L2 req | L2 hit | HBM rd req | L1->L2 rd | L1->L2 wr | rd req/inst |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    m = lambda ent, c: (sum(ent["vals"][c]) / len(ent["vals"][c])) if ent["vals"].get(c) else None
    f = lambda v, fmt: "-" if v is None else format(v, fmt)
    for name, (grid, ent) in sorted(tab.items()):
        if args.kernel and args.kernel not in name:
            continue
        g = m(ent, "GRBM_GUI_ACTIVE")
        cyc = g / XCDS if g else None
        wc = m(ent, "SQ_WAVE_CYCLES")
        wpc = 4 * wc / (cyc * args.cus) if (wc and cyc) else None
        frac = lambda c: (m(ent, c) / wc) if (wc and m(ent, c) is not None) else None
        req, hit = m(ent, "TCC_REQ_sum"), m(ent, "TCC_HIT_sum")
        rd = m(ent, "TCP_TCC_READ_REQ_sum")
        dur = sorted(ent["dur"])[len(ent["dur"]) // 2] / 1e3 if ent.get("dur") else None
        meta = ent["meta"]
        lines.append(
            f"| `{_short(name)}` | {grid} | {2 * meta[2]} | {meta[3]} | {f(dur, '.1f')} | "
            f"{f(wpc, '.1f')} | {f(frac('SQ_WAIT_ANY'), '.2f')} | {f(frac('SQ_WAIT_INST_ANY'), '.2f')} | "
            f"{f(frac('SQ_ACTIVE_INST_ANY'), '.2f')} | {f(req, '.3g')} | "
            f"{f(None if not req else hit / req, '.2f')} | {f(m(ent, 'TCC_EA0_RDREQ_sum'), '.3g')} | "
            f"{f(rd, '.3g')} | {f(m(ent, 'TCP_TCC_WRITE_REQ_sum'), '.3g')} | "
            f"{f(None if rd is None else rd / args.instances, '.0f')} |")
    lines += ["", "VGPR is the allocation the trace reports (twice its VGPR_Count field, the "
              "granule this device counts in); durations are medians under counter collection."]
    with open(args.out, "w") as fh:
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
    s.add_argument("--by-grid", action="store_true",
                   help="one row per kernel and launch size, from the kernel trace")
    s.add_argument("--kernel", default="", help="name fragment of the kernels to list")
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
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--out", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="rocprofv3 counters")
    c.add_argument("--kernel", default="k_eval")
    c.add_argument("--instances", type=int, default=1)
    c.add_argument("--cus", type=int, default=256)
    args = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters}[args.what](args)


if __name__ == "__main__":
    main()
