"""rocprofv3 runs and summaries for the library's kernels on the bench workloads.

Collect every profile the bench relies on (kernel trace, then FETCH_SIZE and WRITE_SIZE
counter passes of their own) and write one summary per kernel:

    python -m paper_1803_00437_amd.profiling collect --raw OUT_DIR --out profiles

Summarise an existing set of rocprofv3 directories (``--output-format csv``) for one kernel:

    python -m paper_1803_00437_amd.profiling summarise --trace DIR [--fetch DIR --write DIR] \\
        --kernel "fd_sweep_kernel<float, 4, 3, false, false, 0>" --launch-alg-bytes 1610612736 \\
        --out profiles/NAME.md [--json profiles/NAME.json --sources a.hip b.hpp]

The HBM counters are scaled by what they read for the library's streaming copy kernel
(``fdlbm_device_copy``), which reads and writes a known number of bytes; the scale factors
are printed with each summary.  This module never touches the GPU itself: rocprofv3 runs
the bench as a child process.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import shutil
import subprocess
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = "paper_1803_00437_amd/csrc"
FD_SOURCES = [f"{CSRC}/fd_sweep.hip", f"{CSRC}/fd_sweep_body.hpp", f"{CSRC}/fdlbm_device.hpp"]
MRT_SOURCES = [f"{CSRC}/mrt.hip", f"{CSRC}/fdlbm_device.hpp"]
D3_SOURCES = [f"{CSRC}/fd3d.hip", f"{CSRC}/fd3d_device.hpp", f"{CSRC}/fdlbm_device.hpp", f"{CSRC}/fd_sweep_body.hpp"]
N3 = 512
COPY_BYTES = 1 << 30
N = 8192
CHANNEL = 16384 * 1024
BATCH_NODES = 177708266  # sum of N^2 over the 512 shear-wave instances (sizes U{32..1024}, seed 5)
# the disk of radius N/2 - 6 centred at ((N-1)/2, (N-1)/2): its ghost nodes (within
# Chebyshev distance 3 of the fluid) and the ring of rest nodes within 3 of those.  A fill
# reads 4 fluid nodes and a 32-byte table entry and writes 1 node per ghost (92 bytes in
# FP32), and reads a 4-byte index and writes 1 node per ring node (16 bytes).
DISK_GHOSTS, DISK_RING = 98196, 98268
DISK_FILL_BYTES = 92 * DISK_GHOSTS + 16 * DISK_RING


def _csvs(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def kernel_stats(d):
    rows = []
    for p in _csvs(d, "kernel_stats.csv"):
        rows += list(csv.DictReader(open(p)))
    return rows


def counter_means(d, counter):
    """{kernel name: (dispatches, mean value of `counter`)} of a --pmc run."""
    acc = defaultdict(list)
    for p in _csvs(d, "counter_collection.csv"):
        for r in csv.DictReader(open(p)):
            if r["Counter_Name"] == counter:
                acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def launch_gaps(d, pattern):
    """Idle time between the dispatches of a replayed sequence: over the window from the
    first to the last dispatch whose kernel name contains `pattern`, the span, the time at
    least one kernel ran (union of the dispatch intervals) and the dispatch count."""
    rows = []
    for p in _csvs(d, "kernel_trace.csv"):
        for r in csv.DictReader(open(p)):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    idx = [i for i, r in enumerate(rows) if pattern in r[2]]
    if not idx:
        return None
    win = rows[idx[0]:idx[-1] + 1]
    busy, cur_s, cur_e = 0, None, None
    for s0, e0, _ in win:
        if cur_e is None or s0 > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    busy += cur_e - cur_s
    span = win[-1][1] - win[0][0]
    return {"span_ns": span, "busy_ns": busy, "dispatches": len(win), "matching": len(idx),
            "idle_frac": 1.0 - busy / span}


def pick(table, pattern):
    hits = [k for k in table if pattern in k]
    if not hits:
        raise SystemExit(f"no kernel matches {pattern!r}")
    return hits[0]


def sources_sha(paths, root=ROOT):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(root, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def summarise(trace, kernel, alg, out_md, *, fetch=None, write=None, json_out=None, sources=(), command="",
              counter_command="", workload="", n=N, copy_kernel="copy_kernel", copy_bytes=COPY_BYTES, generator="",
              group=False):
    """group=True: every kernel matching `kernel` is launched once per unit of work (the
    batched step launches one kernel per lane-width class); their average durations add up
    to the unit's time and `alg` is the bytes of the whole unit."""
    stats = kernel_stats(trace)
    names = {r["Name"]: r for r in stats}
    if group:
        hits = sorted(k for k in names if kernel in k)
        if not hits:
            raise SystemExit(f"no kernel matches {kernel!r}")
        kname = " + ".join(hits)
        k = {"Calls": str(min(int(names[h]["Calls"]) for h in hits))}
        avg_ns = sum(float(names[h]["AverageNs"]) for h in hits)
    else:
        kname = pick(names, kernel)
        k = names[kname]
        avg_ns = float(k["AverageNs"])
    lines = [f"# rocprofv3 summary: `{kernel}`", ""]
    if generator:
        lines += [f"Written by: `{generator}` (runs the commands below on the GPU, then summarises)", ""]
    if workload:
        lines += [f"Workload: {workload}", ""]
    lines += [f"Command (kernel trace): `{command}`", "",
              "| kernel | calls | average ns | min ns | max ns |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
        lines.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | {r['MaxNs']} |")
    lines += ["", f"Summarised kernel: `{kname}`", f"- calls: {k['Calls']}",
              f"- average duration: {avg_ns:.0f} ns" + (" (sum of the kernels' averages: one launch of each per step)"
                                                        if group else ""),
              f"- algorithmic bytes per launch: {alg} ({alg / avg_ns:.1f} GB/s at the average duration, "
              f"{alg / avg_ns / 8000:.3f} of 8 TB/s)"]
    out = {"kernel": kname, "avg_ns": avg_ns, "calls": int(k["Calls"]), "alg_bytes_per_launch": alg, "n": n,
           "alg_gbs": alg / avg_ns}
    if group:
        g = launch_gaps(trace, kernel)
        if g:
            lines += [f"- replayed sequence (first to last `{kernel}` dispatch): {g['dispatches']} dispatches "
                      f"({g['matching']} of them step kernels) over {g['span_ns'] / 1e6:.3f} ms, a kernel running "
                      f"{g['busy_ns'] / 1e6:.3f} ms of it: {100 * g['idle_frac']:.2f} % idle between dispatches"]
            out["launch_gaps"] = g
    if fetch and write:
        fm, wm = counter_means(fetch, "FETCH_SIZE"), counter_means(write, "WRITE_SIZE")
        kf, kw = fm[pick(fm, kernel)], wm[pick(wm, kernel)]
        cf, cw = fm[pick(fm, copy_kernel)], wm[pick(wm, copy_kernel)]
        f_fetch = copy_bytes / 1024.0 / cf[1]
        f_write = copy_bytes / 1024.0 / cw[1]
        fetch_b = kf[1] * 1024 * f_fetch
        write_b = kw[1] * 1024 * f_write
        lines += ["", f"Counter commands: `{counter_command}`", "",
                  "| counter | copy kernel KiB/dispatch | scale (known bytes / counter) | kernel KiB/dispatch | kernel bytes (scaled) |",
                  "|---|---|---|---|---|",
                  f"| FETCH_SIZE | {cf[1]:.1f} | {f_fetch:.4f} | {kf[1]:.1f} | {fetch_b:.4g} |",
                  f"| WRITE_SIZE | {cw[1]:.1f} | {f_write:.4f} | {kw[1]:.1f} | {write_b:.4g} |",
                  "", f"- HBM bytes per launch (scaled counters): {fetch_b + write_b:.4g} "
                  f"= {(fetch_b + write_b) / alg:.3f} x algorithmic "
                  f"(reads {fetch_b / (alg / 2):.3f} x, writes {write_b / (alg / 2):.3f} x)",
                  f"- counter bandwidth at the average duration: {(fetch_b + write_b) / avg_ns:.1f} GB/s"]
        out.update(fetch_bytes_per_launch=fetch_b, write_bytes_per_launch=write_b,
                   hbm_bytes_per_launch=fetch_b + write_b, fetch_scale=f_fetch, write_scale=f_write,
                   copy_kernel=pick(fm, copy_kernel), copy_bytes=copy_bytes)
    if sources:
        out["kernel_source_sha"] = sources_sha(sources)
        out["sources"] = list(sources)
        lines += ["", f"Kernel sources {list(sources)} sha256[:16] = {out['kernel_source_sha']}"]
    out["command"] = command
    out["counter_command"] = counter_command
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    if json_out:
        with open(json_out, "w") as f:
            json.dump(out, f, indent=1)
    return out


# --- collect -----------------------------------------------------------------------------

BENCH = "/root/repo/bench.py"
# default tile shapes (no tuning launches mixed into the averages)
# the bench's own step counts: the first few dozen launches after a pause run up to 25 % slower
# (clock ramp), so a short trace overstates the steady kernel time
TRACE_ARGS = ["--steps", "1000", "--warmup", "50", "--no-cpu", "--copy-probe", "--no-autotune"]
FD_COUNTER_ARGS = ["--steps", "20", "--warmup", "2", "--no-cpu", "--no-compare", "--no-batch", "--copy-probe",
                   "--no-autotune"]
MRT_COUNTER_ARGS = ["--only", "mrt_f32", "--steps", "20", "--warmup", "2", "--copy-probe", "--no-autotune"]
D3_COUNTER_ARGS = ["--only", "d3_f32", "--d3-steps", "20", "--copy-probe"]

# VALU passes (one rocprofv3 --pmc run each): instructions issued and cycles the SIMDs spent
# issuing them, per dispatch of the step kernel
VALU_COUNTERS = ["SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE", "SQ_WAVES"]
VALU_SOURCES = {"fd3_f32": FD_SOURCES, "fd3_f16": FD_SOURCES, "mrt_f32": MRT_SOURCES,
                "batch512": [f"{CSRC}/fd_batch.hip", f"{CSRC}/fd_sweep_body.hpp", f"{CSRC}/fdlbm_device.hpp"],
                "d3_f32": D3_SOURCES}
VALU_PASSES = [
    # name, bench arguments, kernel name pattern, nodes updated per dispatch (summed over the
    # matching kernels of one step)
    ("fd3_f32", ["--only", "fd3_f32", "--steps", "20", "--warmup", "2", "--no-autotune"],
     "fd_sweep_kernel<float, 4, 3, false, false, 0>", N * N),
    ("fd3_f16", ["--only", "fd3_f16", "--steps", "20", "--warmup", "2", "--no-autotune"],
     "fd_sweep_kernel<__half, 4, 3, false, false, 0>", N * N),
    ("mrt_f32", ["--only", "mrt_f32", "--steps", "20", "--warmup", "2", "--no-autotune"],
     "mrt_sweep_kernel<float, 4, 0>", N * N),
    ("batch512", ["--only", "batch", "--batch-steps", "20", "--no-autotune"], "fd_batch_kernel<float, ", BATCH_NODES),
    ("d3_f32", ["--only", "d3_f32", "--d3-steps", "20"], "d3_sweep_kernel<float, 12>", N3 ** 3),
]
SIMDS = 1024  # 256 compute units x 4 SIMDs
XCDS = 8

DECAY = "8192 x 8192 periodic decaying flow (modes 0<|k|<=32, max|field| 0.02), nu 0.02"
KERNELS = [
    # file stem, kernel name pattern, algorithmic bytes per launch, counter pair, sources, workload
    # (the batch stem sums its per-class kernels, see summarise(group=True))
    ("fd3_f32_8192", "fd_sweep_kernel<float, 4, 3, false, false, 0>", 24 * N * N, "fd", FD_SOURCES,
     f"{DECAY}; FD-LBM 3-point, FP32 (3 words read + 3 written per node)"),
    ("mrt_f32_8192", "mrt_sweep_kernel<float, 4, 0>", 72 * N * N, "mrt", MRT_SOURCES,
     f"{DECAY}; MRT D2Q9, FP32 (9 words read + 9 written per node)"),
    ("fd3_f64_8192", "fd_sweep_kernel<double, 2, 3, false, false, 0>", 48 * N * N, None, FD_SOURCES,
     f"{DECAY}; FD-LBM 3-point, FP64"),
    ("fd3_f16_8192", "fd_sweep_kernel<__half, 4, 3, false, false, 0>", 12 * N * N, None, FD_SOURCES,
     f"{DECAY}; FD-LBM 3-point, FP16 storage, FP32 arithmetic"),
    ("fd3_f16sr_8192", "fd_sweep_kernel<fdlbm::HalfSR, 4, 3, false, false, 0>", 12 * N * N, None, FD_SOURCES,
     f"{DECAY}; FD-LBM 3-point, FP16 storage rounded stochastically, FP32 arithmetic"),
    ("fd5_f32_8192", "fd_sweep_kernel<float, 4, 5, false, false, 0>", 24 * N * N, None, FD_SOURCES,
     f"{DECAY}; FD-LBM 5-point, FP32"),
    ("lwacm_f32_8192", "fd_sweep_kernel<float, 4, 1, false, false, 0>", 24 * N * N, None, FD_SOURCES,
     f"{DECAY}; LW-ACM (section 1-b), FP32, the same 3 words per node as FD-LBM"),
    ("mrt_f64_8192", "mrt_sweep_kernel<double, 2, 0>", 144 * N * N, None, MRT_SOURCES,
     f"{DECAY}; MRT D2Q9, FP64"),
    ("fd3_f32_channel_16384x1024", "fd_sweep_kernel<float, 4, 3, true, true, 0>", 24 * CHANNEL, None, FD_SOURCES,
     "Poiseuille channel 16384 x 1024, walls at y=-1/2 and ny-1/2, body force; FD-LBM 3-point, FP32"),
    ("mrt_f32_channel_16384x1024", "mrt_sweep_kernel<float, 4, 1>", 72 * CHANNEL, None, MRT_SOURCES,
     "Poiseuille channel 16384 x 1024, halfway bounce-back walls, body force; MRT D2Q9, FP32"),
    ("fd3_f32_batch512", "fd_batch_kernel<float, ", 24 * BATCH_NODES, None,
     [f"{CSRC}/fd_batch.hip", f"{CSRC}/fd_sweep_body.hpp", f"{CSRC}/fdlbm_device.hpp"],
     "512 periodic shear-wave instances N x N, N ~ U{32..1024}, one launch per step for all; FP32"),
    ("fd3d_f32_512", "d3_sweep_kernel<float, 12>", 32 * N3 ** 3, "d3", D3_SOURCES,
     "512^3 periodic decaying flow (modes 0<|k|<=8, max|field| 0.02), nu 0.02; FD-LBM D3Q19 sweep kernel, FP32 "
     "(4 words read + 4 written per node)"),
    ("fd3d_f64_512", "d3_sweep_kernel<double, 12>", 64 * N3 ** 3, None, D3_SOURCES,
     "512^3 periodic decaying flow (modes 0<|k|<=8, max|field| 0.02), nu 0.02; FD-LBM D3Q19 sweep kernel, FP64"),
    ("disk_fill_f32_8192", "disk_fill_kernel<float>", DISK_FILL_BYTES, None, [f"{CSRC}/disk.hip"],
     "disk of radius 4090 in the 8192 x 8192 grid (section 3-b curved wall): ghost nodes and the ring of rest "
     "nodes set before each FD-LBM 3-point FP32 step (the first fill after the state is set clears every rest "
     "node and is in the average); algorithmic bytes = 92 per ghost + 16 per ring node"),
    ("copy_1gib", "copy_kernel", 2 * COPY_BYTES, None, [f"{CSRC}/diag.hip"],
     "fdlbm_device_copy of 1 GiB (the achievable-bandwidth probe)"),
]


def _run(cmd, log, limit, kill_signal):
    print("+", " ".join(cmd), flush=True)
    with open(log, "w") as f:
        rc = subprocess.call(["timeout", "-s", kill_signal, "-k", "10", str(limit)] + cmd, stdout=f,
                             stderr=subprocess.STDOUT, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"))
    if rc != 0:
        sys.stdout.write(open(log).read()[-3000:])
        raise SystemExit(f"step failed with exit status {rc}: {' '.join(cmd)}")


def valu_summary(raw, out_md, command):
    """VALU busy of each pass: SQ_ACTIVE_INST_VALU x 4 cycles (a wave64 VALU instruction holds
    a SIMD for 4 cycles; packed FP32 is not used) over the SIMD-cycles of the dispatch
    (GRBM_GUI_ACTIVE is summed over the XCDs), and VALU instructions per node update
    (SQ_INSTS_VALU x 64 lanes / nodes)."""
    lines = ["# rocprofv3 VALU counters of the step kernels", "",
             "Written by: `python -m paper_1803_00437_amd.profiling collect --raw <dir> --out profiles`", "",
             "Commands (one counter pass each, nothing else collected):", ""]
    rows = []
    for name, args, pattern, nodes in VALU_PASSES:
        d = os.path.join(raw, f"valu_{name}")
        lines.append(f"    {command} -d <dir>/valu_{name} -- python3 -u {BENCH} " + " ".join(args))
        means = {c: counter_means(d, c) for c in VALU_COUNTERS}
        hits = sorted(k for k in means["SQ_INSTS_VALU"] if pattern in k)
        if not hits:
            raise SystemExit(f"no kernel matches {pattern!r} in {d}")
        insts = sum(means["SQ_INSTS_VALU"][k][1] for k in hits)
        active = sum(means["SQ_ACTIVE_INST_VALU"][k][1] for k in hits)
        cycles = sum(means["GRBM_GUI_ACTIVE"][k][1] for k in hits) / XCDS
        waves = sum(means["SQ_WAVES"][k][1] for k in hits)
        calls = min(means["SQ_INSTS_VALU"][k][0] for k in hits)
        busy = active * 4 / (SIMDS * cycles)
        rows.append((pattern if len(hits) == 1 else pattern + " (" + str(len(hits)) + " kernels per step)", calls,
                     insts, active, cycles * XCDS, waves, busy, insts * 64 / nodes))
    lines += ["", "Per dispatch of the step kernel (per step, summed over its kernels, for the batch), averaged "
              "over the dispatches. VALU busy = SQ_ACTIVE_INST_VALU x 4 / (1024 SIMDs x GRBM_GUI_ACTIVE / 8); "
              "per node = SQ_INSTS_VALU x 64 / nodes updated.", "",
              "| kernel | dispatches | SQ_INSTS_VALU | SQ_ACTIVE_INST_VALU | GRBM_GUI_ACTIVE (sum of 8 XCDs) | "
              "SQ_WAVES | VALU busy | VALU instructions per node |", "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r[0]}` | {r[1]} | {r[2]:.4g} | {r[3]:.4g} | {r[4]:.4g} | {r[5]:.0f} | {100 * r[6]:.0f} % | "
                     f"{r[7]:.1f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    summary = {name: {"kernel": r[0], "valu_insts": r[2], "busy": r[6], "insts_per_node": r[7],
                      "kernel_source_sha": sources_sha(VALU_SOURCES[name])}
               for (name, _, _, _), r in zip(VALU_PASSES, rows)}
    with open(os.path.splitext(out_md)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    return rows


def collect(raw, out, run=True):
    """run=False only rewrites the summaries from rocprofv3 output already in `raw`."""
    raw = os.path.abspath(raw)
    os.makedirs(raw, exist_ok=True)
    os.makedirs(out, exist_ok=True)
    py = ["python3", "-u", BENCH]
    trace_opts = ["--kernel-trace", "--stats", "--output-format", "csv"]
    if run:
        # rocprofv3 names its files by process id: start from empty directories so that no
        # earlier run's files are summarised with this one's
        for sub in ("trace", "fd_fetch_size", "fd_write_size", "mrt_fetch_size", "mrt_write_size", "d3_fetch_size",
                    "d3_write_size") + tuple(
                f"valu_{p[0]}" for p in VALU_PASSES):
            shutil.rmtree(os.path.join(raw, sub), ignore_errors=True)
        _run(["rocprofv3"] + trace_opts + ["-d", f"{raw}/trace", "--"] + py + TRACE_ARGS, f"{raw}/trace.log", 400,
             "TERM")
    pmc = {}
    for name, args in (("fd", FD_COUNTER_ARGS), ("mrt", MRT_COUNTER_ARGS), ("d3", D3_COUNTER_ARGS)):
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            d = f"{raw}/{name}_{counter.lower()}"
            if run:
                _run(["rocprofv3", "--pmc", counter, "--output-format", "csv", "-d", d, "--"] + py + args,
                     f"{d}.log", 120, "KILL")
        pmc[name] = (f"{raw}/{name}_fetch_size", f"{raw}/{name}_write_size",
                     f"cd /tmp && TMPDIR=/tmp rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv "
                     f"-d <dir> -- python3 -u {BENCH} " + " ".join(args))
    valu_cmd = ["rocprofv3", "--pmc"] + VALU_COUNTERS + ["--output-format", "csv"]
    if run:
        for name, args, _, _ in VALU_PASSES:
            d = f"{raw}/valu_{name}"
            _run(valu_cmd + ["-d", d, "--"] + py + args, f"{d}.log", 120, "KILL")
    valu = valu_summary(raw, os.path.join(out, "valu_busy_8192.md"), "cd /tmp && TMPDIR=/tmp " + " ".join(valu_cmd))
    for r in valu:
        print(f"valu {r[0]}: {r[2]:.4g} instructions, {100 * r[6]:.0f} % busy, {r[7]:.1f} per node")
    trace_str = "cd /tmp && TMPDIR=/tmp " + " ".join(["rocprofv3"] + trace_opts + ["-d", "<dir>", "--"] + py + TRACE_ARGS)
    results = {}
    for stem, pattern, alg, counters, sources, workload in KERNELS:
        kw = {}
        if counters:
            f, w, cc = pmc[counters]
            kw = dict(fetch=f, write=w, counter_command=cc, json_out=os.path.join(out, f"{stem}_counters.json"))
        results[stem] = summarise(f"{raw}/trace", pattern, alg, os.path.join(out, f"{stem}.md"), sources=sources,
                                  command=trace_str, workload=workload, group=stem.endswith("batch512"),
                                  n=N3 if stem.startswith("fd3d") else N,
                                  generator="python -m paper_1803_00437_amd.profiling collect --raw <dir> --out profiles",
                                  **kw)
        r = results[stem]
        print(f"{stem}: {r['avg_ns']:.0f} ns, {r['alg_gbs']:.0f} GB/s algorithmic"
              + (f", HBM {r['hbm_bytes_per_launch'] / alg:.3f} x algorithmic" if "hbm_bytes_per_launch" in r else ""))
    print(f"(regenerate: python -m paper_1803_00437_amd.profiling collect --raw {raw} --out {out})")
    return results


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect", help="run rocprofv3 on the bench and write every summary")
    c.add_argument("--raw", required=True, help="directory for rocprofv3 output (large; not for committing)")
    c.add_argument("--out", required=True, help="directory for the summaries")
    c.add_argument("--summaries-only", action="store_true", help="rewrite the summaries from existing output")
    s = sub.add_parser("summarise", help="summarise existing rocprofv3 output for one kernel")
    s.add_argument("--trace", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--kernel", required=True, help="substring of the kernel name to summarise")
    s.add_argument("--launch-alg-bytes", type=int, required=True, help="algorithmic bytes moved per launch")
    s.add_argument("--command", default="")
    s.add_argument("--counter-command", default="")
    s.add_argument("--out", required=True)
    s.add_argument("--json")
    s.add_argument("--sources", nargs="*", default=[])
    s.add_argument("--n", type=int, default=N)
    args = ap.parse_args()
    if args.cmd == "collect":
        collect(args.raw, args.out, run=not args.summaries_only)
    else:
        summarise(args.trace, args.kernel, args.launch_alg_bytes, args.out, fetch=args.fetch, write=args.write,
                  json_out=args.json, sources=args.sources, command=args.command,
                  counter_command=args.counter_command, n=args.n)
        print(open(args.out).read())


if __name__ == "__main__":
    main()
