"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1803_00437_amd.profiling \\
        --trace DIR [--fetch DIR --write DIR] --kernel fd_sweep_kernel<float \\
        --copy-bytes 1073741824 --launch-alg-bytes 1610612736 --command "..." \\
        --out profiles/NAME.md [--json profiles/NAME.json --sources a.hip b.hpp]

DIR are rocprofv3 output directories written with ``--output-format csv``:
``--kernel-trace --stats`` for the trace, ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` for
the two counter runs.  The counters are scaled by what they read for the library's
streaming copy kernel (``fdlbm_device_copy``), which reads and writes a known number of
bytes; the scale factors are printed with the summary.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict


def _csvs(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def kernel_stats(d):
    rows = []
    for p in _csvs(d, "kernel_stats.csv"):
        rows += list(csv.DictReader(open(p)))
    return rows


def counter_means(d):
    """{kernel name: (dispatches, mean counter value)} of a --pmc run."""
    acc = defaultdict(list)
    for p in _csvs(d, "counter_collection.csv"):
        for r in csv.DictReader(open(p)):
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def pick(table, pattern):
    hits = [k for k in table if pattern in k]
    if not hits:
        raise SystemExit(f"no kernel matches {pattern!r}")
    return hits[0]


def sources_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", required=True, help="substring of the kernel name to summarise")
    ap.add_argument("--copy-kernel", default="copy_kernel")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--launch-alg-bytes", type=int, required=True, help="algorithmic bytes moved per launch")
    ap.add_argument("--command", default="")
    ap.add_argument("--counter-command", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--json")
    ap.add_argument("--sources", nargs="*", default=[])
    ap.add_argument("--n", type=int, default=8192)
    args = ap.parse_args()

    stats = kernel_stats(args.trace)
    names = {r["Name"]: r for r in stats}
    kname = pick(names, args.kernel)
    k = names[kname]
    avg_ns = float(k["AverageNs"])
    lines = [f"# rocprofv3 summary: {args.kernel}", "",
             f"Command (kernel trace): `{args.command}`", ""]
    lines += ["| kernel | calls | average ns | min ns | max ns |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        lines.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | {r['MaxNs']} |")
    alg = args.launch_alg_bytes
    lines += ["", f"Summarised kernel: `{kname}`", f"- average duration: {avg_ns:.0f} ns",
              f"- algorithmic bytes per launch: {alg} ({alg / avg_ns:.1f} GB/s at the average duration)"]
    out = {"kernel": kname, "avg_ns": avg_ns, "alg_bytes_per_launch": alg, "n": args.n}
    if args.fetch and args.write:
        fm, wm = counter_means(args.fetch), counter_means(args.write)
        kf, kw = fm[pick(fm, args.kernel)], wm[pick(wm, args.kernel)]
        cf, cw = fm[pick(fm, args.copy_kernel)], wm[pick(wm, args.copy_kernel)]
        f_fetch = args.copy_bytes / 1024.0 / cf[1]
        f_write = args.copy_bytes / 1024.0 / cw[1]
        fetch_b = kf[1] * 1024 * f_fetch
        write_b = kw[1] * 1024 * f_write
        lines += ["", f"Counter commands: `{args.counter_command}`", "",
                  "| counter | copy kernel KiB/dispatch | scale (known bytes / counter) | kernel KiB/dispatch | kernel bytes (scaled) |",
                  "|---|---|---|---|---|",
                  f"| FETCH_SIZE | {cf[1]:.1f} | {f_fetch:.4f} | {kf[1]:.1f} | {fetch_b:.4g} |",
                  f"| WRITE_SIZE | {cw[1]:.1f} | {f_write:.4f} | {kw[1]:.1f} | {write_b:.4g} |",
                  "", f"- HBM bytes per launch (scaled counters): {fetch_b + write_b:.4g} "
                  f"= {(fetch_b + write_b) / alg:.3f} x algorithmic",
                  f"- counter bandwidth at the average duration: {(fetch_b + write_b) / avg_ns:.1f} GB/s"]
        out.update(fetch_bytes_per_launch=fetch_b, write_bytes_per_launch=write_b,
                   hbm_bytes_per_launch=fetch_b + write_b, fetch_scale=f_fetch, write_scale=f_write,
                   copy_kernel=pick(fm, args.copy_kernel), copy_bytes=args.copy_bytes)
    if args.sources:
        out["kernel_source_sha"] = sources_sha(args.sources)
        out["sources"] = args.sources
        lines += ["", f"Kernel sources {args.sources} sha256[:16] = {out['kernel_source_sha']}"]
    out["command"] = args.command
    out["counter_command"] = args.counter_command
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
