#!/usr/bin/env python3
"""Throughput of the FD-LBM D2Q9 step on one MI355X, with the MRT D2Q9 step beside it.

Workload: the 8192 x 8192 periodic decaying flow (random Fourier modes 0<|k|<=32 per field,
max |field| = 0.02, seed 4), FD-LBM with 3-point finite differences, nu = 0.02, s_e = 1,
FP32 storage and arithmetic.  One step is one FD-LBM time step of the whole grid; the
timed region also runs the FP64 diagnostics reduction every 100 steps.

Prints ONE JSON line: value = FD-LBM FP32 MLUPS (million lattice-node updates per
second), the HBM roofline of the step kernel (algorithmic bytes: 3 FP32 words read and 3
written per node), the CPU oracle timed on a bounded band of the same workload, the
relative L2 error of each GPU dtype against that oracle band, and the same measurements
for the MRT step, the FP64 and FP16-storage FD-LBM steps and the 5-point stencil.  The
FD-LBM step on the D3Q19 lattice is timed beside them on a 512^3 periodic decaying flow
(object "d3q19").

    python bench.py [--steps K] [--warmup W] [--n 8192] [--no-compare] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM peak, FD-LBM vs MRT D2Q9 at 8192² FP32 (err vs FP64 oracle)"
HBM_PEAK_GBS = 8000.0
NU = 0.02
DIAG_EVERY = 100
COUNTERS = os.path.join(ROOT, "profiles", "fd3_f32_8192_counters.json")


def kernel_source_sha():
    """Hash of the FD step kernel's sources: counters taken on other sources are not reported."""
    from paper_1803_00437_amd.profiling import FD_SOURCES, sources_sha

    return sources_sha(FD_SOURCES, ROOT)


def bytes_per_node(scheme, dtype):
    words = 9 if scheme == "mrt" else 3
    return 2 * words * {"f64": 8, "f32": 4, "f16": 2, "f16sr": 2}[dtype]


def run_case(F, torch, init, scheme, dtype, stencil, steps, warmup, kernel, with_diag, tile_rows=0, lane_cols=0,
             bc="periodic", nu=NU, force=(0.0, 0.0), autotune=True, disk=(0.0, 0.0, 0.0)):
    ny, nx = init[0].shape
    s_xx = F.fdlbm_rate_from_viscosity(nu)
    kw = dict(scheme=scheme, dtype=dtype, s_xx=s_xx, s_e=1.0, kernel=kernel, tile_rows=tile_rows, bc=bc, force=force,
              disk=disk)
    if scheme != "mrt":
        kw["lane_cols"] = lane_cols
    if scheme == "fd":
        kw["stencil"] = stencil
    elif scheme == "mrt":
        kw["quartic"] = True
    sim = F.FdLbm(nx, ny, **kw)
    sim.set_state(*init)
    shape = None
    if autotune and not (tile_rows or lane_cols):
        # tile shape picked by the library's tuner on this grid (untimed set-up)
        shape = sim.autotune(reps=10)[:2]
    sim.step(warmup)
    torch.cuda.synchronize()
    # kernel-only region, timed with HIP events on the library's stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    e1.synchronize()
    kernel_ms = e0.elapsed_time(e1) / steps
    # whole-step region (steps + periodic diagnostics), wall clock between synchronisations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(DIAG_EVERY, steps - done)
        sim.step(k)
        done += k
        if with_diag:
            sim.diagnostics()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    diag = sim.diagnostics()
    sim.close()
    nodes = nx * ny
    return {
        "ms_per_step": wall_ms,
        "kernel_ms": kernel_ms,
        "mlups": nodes / (wall_ms * 1e3),
        "kernel_mlups": nodes / (kernel_ms * 1e3),
        "alg_gbs": bytes_per_node(scheme, dtype) * nodes / (kernel_ms * 1e6),
        "nonfinite": diag["nonfinite"],
        "tile": {"lane_cols": shape[0], "tile_rows": shape[1]} if shape else None,
    }


D3_N = 512
VALU_JSON = os.path.join(ROOT, "profiles", "valu_busy_8192.json")
# issue rate of FP32 vector instructions without packed math: 256 compute units x 4 SIMDs x
# 16 lanes per cycle (a wave64 instruction holds a SIMD for 4 cycles) x 2.4 GHz
VALU_PEAK = 256 * 4 * 16 * 2.4e9


def d3_alu_roofline(kernel_ms, nodes):
    """The D3Q19 sweep is bound by instruction issue: VALU lane-instructions per second against
    the chip's issue rate, with the instructions per node the rocprofv3 VALU pass measured on
    the same kernel sources (None when the counters were taken on other sources)."""
    if not os.path.exists(VALU_JSON):
        return None
    from paper_1803_00437_amd.profiling import VALU_SOURCES, sources_sha

    with open(VALU_JSON) as f:
        v = json.load(f).get("d3_f32")
    if not v or v.get("kernel_source_sha") != sources_sha(VALU_SOURCES["d3_f32"], ROOT):
        return None
    achieved = v["insts_per_node"] * nodes / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK, "unit": "VALU lane-instructions/s",
            "frac": achieved / VALU_PEAK, "insts_per_node": v["insts_per_node"], "valu_busy_counter": v["busy"]}
D3_WORKLOAD = ("{n}^3 periodic decaying flow, random Fourier modes 0<|k|<=8 per field, max|field|=0.02, seed 6; "
               "FD-LBM D3Q19 3-point finite differences, nu=0.02, s_e=1")


def d3_bytes_per_node(dtype):
    return 2 * 4 * {"f64": 8, "f32": 4}[dtype]


def run_d3(F, torch, init, dtype, steps, warmup):
    """The FD-LBM step on the D3Q19 lattice (fused sweep kernel, default tile), timed with HIP
    events on the library's stream; whole-step time with FP64 diagnostics every 100 steps."""
    nz, ny, nx = init[0].shape
    sim = F.FdLbm3D(nx, ny, nz, dtype=dtype, s_nu=F.fdlbm_rate_from_viscosity(NU), s_e=1.0)
    sim.set_state(*init)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    e1.synchronize()
    kernel_ms = e0.elapsed_time(e1) / steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(DIAG_EVERY, steps - done)
        sim.step(k)
        done += k
        sim.diagnostics()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    diag = sim.diagnostics()
    sim.close()
    nodes = nx * ny * nz
    alg = d3_bytes_per_node(dtype) * nodes / (kernel_ms * 1e6)
    return {
        "ms_per_step": wall_ms,
        "kernel_ms": kernel_ms,
        "mlups": nodes / (wall_ms * 1e3),
        "kernel_mlups": nodes / (kernel_ms * 1e3),
        "alg_gbs": alg,
        "hbm_frac": alg / HBM_PEAK_GBS,
        "nonfinite": diag["nonfinite"],
    }


def d3_oracle_baseline(O3, n=160, steps=3):
    """The FP64 D3Q19 oracle timed on an n^3 periodic sample of the same kind of flow."""
    import workloads as W

    init = W.decaying_flow3(n, seed=6, amp=0.02)
    t0 = time.perf_counter()
    O3.fd3d_run(*init, steps, s_nu=1.0 / (0.5 + 3 * NU), s_e=1.0)
    secs = time.perf_counter() - t0
    return {"value": n ** 3 * steps / secs / 1e6, "unit": "MLUPS", "kind": "oracle",
            "sample": f"FP64 CPU oracle of the D3Q19 step, {steps} steps of a {n}^3 periodic decaying flow "
                      f"({secs:.1f} s)"}


def measure_copy(F, torch, probe=False, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: the library's streaming copy of 1 GiB (read + write)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(5 if probe else 2):
        F.fdlbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        F.fdlbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e6)


def run_batch(F, torch, W, steps, per_instance_steps, every=10, autotune=True):
    """The 512-instance shear-wave sweep: N ~ U{32..1024}, nu ~ U[0.005, 0.1], m ~ U{1..4},
    FP32, 3-point differences; one launch per step for all instances with A(t) sampled every
    `every` steps (graph-replayed), against one launch per instance per step."""
    insts = W.batch_instances(512, seed=5)
    specs = [(d["n"], d["n"], F.fdlbm_rate_from_viscosity(d["nu"]), 1.0) for d in insts]
    b = F.FdLbmBatch(specs, dtype="f32", max_samples=(steps + 20) // every + 1)
    for i, d in enumerate(insts):
        b.set_state(i, *W.shear_wave_y(d["n"], d["n"], d["amp"], d["m"]))
    nodes = sum(d["n"] * d["n"] for d in insts)
    rows = b.autotune(reps=3)[0] if autotune else 8
    b.step(20, sample_every=every, use_graph=True)
    b.stream.synchronize()
    t0 = time.perf_counter()
    b.step(steps, sample_every=every, use_graph=True)
    b.stream.synchronize()
    graph_s = time.perf_counter() - t0
    b.step_per_instance(4)
    b.stream.synchronize()
    t0 = time.perf_counter()
    b.step_per_instance(per_instance_steps)
    b.stream.synchronize()
    single_s = time.perf_counter() - t0
    nsamp = b.amplitudes().shape[1]
    b.close()
    return {
        "instances": len(insts), "nodes": nodes, "sample_every": every, "samples": nsamp, "tile_rows": rows,
        "graph_steps": steps, "graph_ms_per_step": round(graph_s * 1e3 / steps, 4),
        "graph_instance_steps_per_s": round(len(insts) * steps / graph_s, 1),
        "graph_mlups": round(nodes * steps / graph_s / 1e6, 1),
        "per_instance_steps": per_instance_steps,
        "per_instance_ms_per_step": round(single_s * 1e3 / per_instance_steps, 4),
        "per_instance_instance_steps_per_s": round(len(insts) * per_instance_steps / single_s, 1),
        "speedup": round((per_instance_steps and (single_s / per_instance_steps)) / (graph_s / steps), 3),
    }


def band_errors(F, O, init, n, s_steps, rows, cases, threads, cpu_rows):
    """Relative L2 error of each GPU case after s_steps over a band of rows, against the
    FP64 oracle run on that band alone (a band of rows +- the domain of dependence
    s_steps * (h + 1) rows, periodic in y, whose contaminated edges are discarded).  The
    3-point FD-LBM band is cpu_rows tall (when taller than rows): its oracle run is the
    timed CPU baseline, and its first rows give the error."""
    import numpy as np

    y0 = n // 3
    out = {}
    oracle_time = None
    O.num_threads(threads)
    s_xx = F.fdlbm_rate_from_viscosity(NU)
    refs = {}
    for scheme, stencil in sorted({(c[0], c[2]) for c in cases}):
        m = s_steps * ((2 if stencil == 3 else 3) if scheme == "fd" else 1)
        height = max(rows, min(cpu_rows, n - y0 - m)) if (scheme, stencil) == ("fd", 3) else rows
        sl = slice(y0 - m, y0 + height + m)
        band = tuple(np.ascontiguousarray(a[sl]) for a in init)
        t0 = time.perf_counter()
        if scheme == "fd":
            res = O.fd_run(*band, s_steps, s_xx=s_xx, s_e=1.0, stencil=stencil)
        elif scheme == "lwacm":
            res = O.lwacm_run(*band, s_steps, nu=NU)
        else:
            res = O.mrt_moments(O.mrt_run(O.mrt_init(*band), s_steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx)))
        dt = time.perf_counter() - t0
        if scheme == "fd" and stencil == 3:
            oracle_time = (band[0].size * s_steps, dt, band[0].shape[0])
        refs[(scheme, stencil)] = tuple(a[m:m + rows] for a in res)
    for scheme, dtype, stencil in cases:
        kw = dict(scheme=scheme, dtype=dtype, s_xx=s_xx, s_e=1.0)
        kw.update({"stencil": stencil} if scheme == "fd" else {"quartic": True} if scheme == "mrt" else {})
        sim = F.FdLbm(n, n, **kw)
        sim.set_state(*init)
        sim.step(s_steps)
        got = sim.get_state()
        sim.close()
        want = refs[(scheme, stencil)]
        num = sum(float(np.sum((g[y0:y0 + rows] - w) ** 2)) for g, w in zip(got, want))
        den = sum(float(np.sum(w * w)) for w in want)
        out[f"{scheme}{stencil if scheme == 'fd' else ''}_{dtype}"] = math.sqrt(num / den)
    return out, oracle_time


def host_cpus():
    """What the host offers: logical CPUs, those this process may run on, and the model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def oracle_single_thread(F, O, init, n, s_steps, rows):
    """The FP64 oracle on one thread: the 3-point step on a band of `rows` rows (plus the
    domain of dependence) of the same workload, wall clock of the step loop only."""
    import numpy as np

    m = 2 * s_steps
    y0 = n // 3
    band = tuple(np.ascontiguousarray(a[y0 - m:y0 + rows + m]) for a in init)
    O.num_threads(1)
    t0 = time.perf_counter()
    O.fd_run(*band, s_steps, s_xx=F.fdlbm_rate_from_viscosity(NU), s_e=1.0, stencil=3)
    dt = time.perf_counter() - t0
    updates = band[0].size * s_steps
    return {"value": updates / dt / 1e6, "unit": "MLUPS", "cores": O.num_threads(0),
            "sample": f"{s_steps} steps on a {n} x {band[0].shape[0]}-row band "
                      f"({updates / 1e6:.1f} M node updates in {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--kernel", default="auto", choices=["auto", "reference", "sweep"])
    ap.add_argument("--no-compare", action="store_true", help="skip MRT / FP64 / FP16 / 5-point lines")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and error bands")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-instance batch line")
    ap.add_argument("--no-d3", action="store_true", help="skip the D3Q19 lines")
    ap.add_argument("--d3-steps", type=int, default=100)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--err-steps", type=int, default=12)
    ap.add_argument("--err-rows", type=int, default=512)
    ap.add_argument("--cpu-rows", type=int, default=2048,
                    help="rows of the 3-point band whose FP64 oracle run is timed as the CPU baseline")
    ap.add_argument("--cpu-rows-1t", type=int, default=512,
                    help="rows of the band whose FP64 oracle run is timed on one thread")
    ap.add_argument("--tile-rows", type=int, default=0, help="rows per wavefront strip of the sweep kernel (0 = default)")
    ap.add_argument("--lane-cols", type=int, default=0, help="grid columns per lane of the sweep kernel (0 = default)")
    ap.add_argument("--only", default=None,
                    help="time only this case instead of FD3 FP32, e.g. mrt_f32, fd3_f16, lwacm_f32, batch, "
                         "d3_f32 (D3Q19)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default tile shapes instead of tuning them before timing")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run the 1 GiB streaming copy a few more times (calibrates HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the FD-LBM path of this "
              "library has no multi-GPU build (it would split the grid into row bands, each GPU exchanging its edge "
              "rows with its neighbours every step: two for 3-point differences, three for 5-point)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1803_00437_amd as F
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    F.load_library()
    if args.only in ("d3_f32", "d3_f64"):
        copy_gbs = measure_copy(F, torch, probe=args.copy_probe)
        init3 = W.decaying_flow3(D3_N, seed=6, amp=0.02)
        case = run_d3(F, torch, init3, args.only.split("_")[1], args.d3_steps, 5)
        print(json.dumps({"case": args.only, "workload": D3_WORKLOAD.format(n=D3_N), "copy_gbs": copy_gbs, **case}),
              flush=True)
        return
    n = args.n
    t0 = time.perf_counter()
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    print(f"# input {n}x{n} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    copy_gbs = measure_copy(F, torch, probe=args.copy_probe)
    print(f"# streaming copy (fdlbm_device_copy, 1 GiB): {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)

    if args.only == "batch":
        batch = run_batch(F, torch, W, args.batch_steps, max(10, args.batch_steps // 4), autotune=not args.no_autotune)
        print(json.dumps({"case": "batch", **batch}), flush=True)
        return
    if args.only:
        name, dtype = args.only.split("_")
        scheme = name if name in ("mrt", "lwacm") else "fd"
        stencil = int(name[2]) if scheme == "fd" else 0
        case = run_case(F, torch, init, scheme, dtype, stencil, args.steps, args.warmup, args.kernel, False,
                        args.tile_rows, args.lane_cols, autotune=not args.no_autotune)
        print(json.dumps({"case": args.only, "tile_rows": args.tile_rows, "lane_cols": args.lane_cols, **case}),
              flush=True)
        return

    main_case = run_case(F, torch, init, "fd", "f32", 3, args.steps, args.warmup, args.kernel, True,
                         args.tile_rows, args.lane_cols, autotune=not args.no_autotune)
    print(f"# fd3 f32: {main_case}", file=sys.stderr, flush=True)

    compare = {}
    if not args.no_compare:
        short = max(100, args.steps // 4)
        for scheme, dtype, stencil in (("mrt", "f32", 0), ("fd", "f64", 3), ("fd", "f16", 3), ("fd", "f16sr", 3),
                                       ("fd", "f32", 5), ("mrt", "f64", 0), ("lwacm", "f32", 0)):
            key = f"{scheme}{stencil if scheme == 'fd' else ''}_{dtype}"
            compare[key] = run_case(F, torch, init, scheme, dtype, stencil, short, args.warmup, args.kernel, False,
                                    autotune=not args.no_autotune)
            print(f"# {key}: {compare[key]}", file=sys.stderr, flush=True)
        # the 16384 x 1024 Poiseuille channel: walls at y = -1/2 and ny - 1/2, body force along x
        nu_ch = 1.0 / math.sqrt(108.0)
        r, x, y, fx = W.poiseuille_profile(16384, 1024, nu_ch, 0.05)
        for scheme, stencil in (("fd", 3), ("mrt", 0)):
            key = f"poiseuille_16384x1024_{scheme}{stencil if scheme == 'fd' else ''}_f32"
            compare[key] = run_case(F, torch, (r, x, y), scheme, "f32", stencil, short, args.warmup, args.kernel,
                                    False, bc="walls", nu=nu_ch, force=(fx, 0.0), autotune=not args.no_autotune)
            print(f"# {key}: {compare[key]}", file=sys.stderr, flush=True)
        del r, x, y
        # a disk of radius n/2 - 6 closed by the curved wall (section 3-b): the ghost fill
        # (one launch, in place) before each periodic step; the flow is the decaying one,
        # zero outside the disk
        import numpy as np

        c, rad = (n - 1) / 2, n / 2 - 6
        yy, xx = np.ogrid[:n, :n]
        inside = (xx - c) ** 2 + (yy - c) ** 2 < rad * rad
        dinit = tuple(np.where(inside, a, 0.0) for a in init)
        del inside
        key = f"disk_r{rad:g}_fd3_f32"
        compare[key] = run_case(F, torch, dinit, "fd", "f32", 3, short, args.warmup, args.kernel, False, bc="disk",
                                disk=(c, c, rad), autotune=not args.no_autotune)
        compare[key]["vs_periodic"] = round(compare[key]["kernel_ms"] / main_case["kernel_ms"], 4)
        print(f"# {key}: {compare[key]}", file=sys.stderr, flush=True)
        del dinit

    batch = None
    if not args.no_batch:
        batch = run_batch(F, torch, W, args.batch_steps, max(10, args.batch_steps // 4), autotune=not args.no_autotune)
        print(f"# batch: {batch}", file=sys.stderr, flush=True)

    d3 = None
    if not args.no_d3:
        t0 = time.perf_counter()
        init3 = W.decaying_flow3(D3_N, seed=6, amp=0.02)
        print(f"# input {D3_N}^3 generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        d3 = {"workload": D3_WORKLOAD.format(n=D3_N), "bytes_per_node": {"f32": 32, "f64": 64}}
        for dtype in ("f32", "f64"):
            d3[dtype] = run_d3(F, torch, init3, dtype, args.d3_steps, 5)
            print(f"# d3q19 {dtype}: {d3[dtype]}", file=sys.stderr, flush=True)
        d3["roofline_f32"] = d3_alu_roofline(d3["f32"]["kernel_ms"], D3_N ** 3)
        del init3
        if not args.no_cpu:
            from oracle import d3q19 as O3

            d3["cpu_oracle"] = d3_oracle_baseline(O3)
            print(f"# d3q19 cpu oracle: {d3['cpu_oracle']}", file=sys.stderr, flush=True)

    cpu = None
    errors = None
    if not args.no_cpu:
        import oracle as O

        threads = min(os.cpu_count() or 1, 16)
        cases = [("fd", "f32", 3), ("fd", "f64", 3), ("fd", "f16", 3), ("fd", "f16sr", 3), ("fd", "f32", 5),
                 ("mrt", "f32", 0),
                 ("mrt", "f64", 0), ("lwacm", "f32", 0)]
        errors, (updates, secs, band_rows) = band_errors(F, O, init, n, args.err_steps, args.err_rows, cases, threads,
                                              args.cpu_rows)
        print(f"# errors vs oracle: {errors}", file=sys.stderr, flush=True)
        used = O.num_threads(0)
        one = oracle_single_thread(F, O, init, n, args.err_steps, args.cpu_rows_1t)
        O.num_threads(threads)
        cpu = {
            "value": updates / secs / 1e6,
            "unit": "MLUPS",
            "cores": used,
            "kind": "oracle",
            "sample": f"FP64 CPU oracle, FD-LBM 3-point, {args.err_steps} steps on a {n} x "
                      f"{band_rows}-row band of the {n}x{n} decaying flow "
                      f"({updates / 1e6:.1f} M node updates in {secs:.1f} s, {used} OpenMP threads)",
            "single_thread": one,
            "host": host_cpus(),
        }
        print(f"# cpu baseline: {cpu}", file=sys.stderr, flush=True)

    counters = None
    if os.path.exists(COUNTERS):
        with open(COUNTERS) as f:
            c = json.load(f)
        if c.get("kernel_source_sha") == kernel_source_sha() and c.get("n") == n:
            counters = c
    ms = main_case["ms_per_step"]
    kernel_ms = main_case["kernel_ms"]
    achieved = main_case["alg_gbs"]
    line = {
        "metric": METRIC,
        "value": round(main_case["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n}x{n} periodic decaying flow, random Fourier modes 0<|k|<=32, max|field|=0.02, seed 4; "
                        f"FD-LBM D2Q9 3-point finite differences, nu={NU}, s_e=1, FP32; FP64 diagnostics every "
                        f"{DIAG_EVERY} steps",
            "nx": n, "ny": n, "stencil": 3, "kernel": args.kernel, "tile": main_case["tile"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (round(counters["hbm_bytes_per_launch"] / (kernel_ms * 1e6), 1) if counters else None),
            "traffic_bytes_per_launch": (counters["hbm_bytes_per_launch"] if counters else None),
            "kernel_ms": round(kernel_ms, 5),
            "alg_bytes_per_launch": bytes_per_node("fd", "f32") * n * n,
        },
        "hbm_copy": {"gbs": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                     "kernel_frac_of_copy": round(achieved / copy_gbs, 4),
                     "what": "fdlbm_device_copy of 1 GiB: read + write bytes / time"},
        "cpu_baseline": cpu,
        "err_vs_oracle": errors,
        "batch_512": batch,
        "d3q19": ({k: ({kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                       if isinstance(v, dict) else v) for k, v in d3.items()} if d3 else None),
        "compare": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in compare.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
