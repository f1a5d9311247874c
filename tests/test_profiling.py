"""Host checks of the rocprofv3 summariser: the scaling of the HBM byte counters by the
copy kernel of known traffic, and the constants it uses for the bench workloads."""
import csv
import json
import os

import pytest

from paper_1803_00437_amd import profiling as P


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summary_scales_counters_by_the_copy_kernel(tmp_path):
    trace, fetch, write = (str(tmp_path / d) for d in ("trace", "fetch", "write"))
    _write_csv(os.path.join(trace, "vm", "1_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
               [["void k<float>(int)", 10, 4000000, 400000, 90, 390000, 410000, 1],
                ["copy_kernel(x)", 5, 1500000, 300000, 10, 290000, 310000, 1]])
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    copy_kib = (1 << 30) / 1024
    # the fetch counter reads half of the copy's bytes, the write counter all of them
    _write_csv(os.path.join(fetch, "vm", "1_counter_collection.csv"), hdr,
               [["copy_kernel(x)", "FETCH_SIZE", copy_kib / 2], ["void k<float>(int)", "FETCH_SIZE", 600000.0],
                ["void k<float>(int)", "FETCH_SIZE", 600000.0]])
    _write_csv(os.path.join(write, "vm", "1_counter_collection.csv"), hdr,
               [["copy_kernel(x)", "WRITE_SIZE", copy_kib], ["void k<float>(int)", "WRITE_SIZE", 800000.0]])
    out = P.summarise(trace, "k<float>", 1_600_000_000, str(tmp_path / "s.md"), fetch=fetch, write=write,
                      command="cmd", counter_command="ccmd")
    assert out["avg_ns"] == 400000
    assert out["fetch_scale"] == pytest.approx(2.0)
    assert out["write_scale"] == pytest.approx(1.0)
    assert out["hbm_bytes_per_launch"] == pytest.approx(600000 * 1024 * 2 + 800000 * 1024)
    text = open(tmp_path / "s.md").read()
    assert "cmd" in text and "ccmd" in text and "FETCH_SIZE" in text


def test_batch_node_count_matches_the_workload():
    import workloads as W

    assert P.BATCH_NODES == sum(d["n"] ** 2 for d in W.batch_instances(512, seed=5))


def test_kernel_sources_exist():
    for _, _, _, _, sources, _ in P.KERNELS:
        for s in sources:
            assert os.path.exists(os.path.join(P.ROOT, s)), s


def test_bench_refuses_more_than_one_gpu():
    """The step runs on one GPU: bench.py --gpus N with N > 1 exits with a message before it
    touches a device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_launch_gaps_of_a_replayed_sequence(tmp_path):
    """The idle share between dispatches is measured from the first to the last dispatch of
    the step kernel: overlapping dispatches count once, the gaps between them count as idle."""
    trace = str(tmp_path / "trace")
    _write_csv(os.path.join(trace, "vm", "1_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [["other", 0, 50], ["fd_batch_kernel<float, 4, 0>", 100, 200], ["fd_batch_kernel<float, 4, 2>", 210, 400],
                ["proj_partials<float>", 390, 420], ["fd_batch_kernel<float, 4, 0>", 500, 600], ["other", 700, 800]])
    g = P.launch_gaps(trace, "fd_batch_kernel")
    assert g["span_ns"] == 500 and g["busy_ns"] == 100 + 210 + 100 and g["dispatches"] == 4 and g["matching"] == 3
    assert g["idle_frac"] == pytest.approx(1 - 410 / 500)


def test_valu_summary_busy_and_instructions_per_node(tmp_path):
    """VALU busy = SQ_ACTIVE_INST_VALU x 4 / (1024 SIMDs x GRBM_GUI_ACTIVE / 8), and the
    instructions per node = SQ_INSTS_VALU x 64 / nodes; the batch sums its class kernels."""
    raw = str(tmp_path)
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    for name, args, pattern, nodes in P.VALU_PASSES:
        kernels = [pattern + "0>", pattern + "2>"] if name == "batch512" else [pattern]
        rows = []
        for k in kernels:
            rows += [[k, "SQ_INSTS_VALU", 1e8], [k, "SQ_ACTIVE_INST_VALU", 2e8],
                     [k, "GRBM_GUI_ACTIVE", 8e6], [k, "SQ_WAVES", 100]]
        _write_csv(os.path.join(raw, f"valu_{name}", "vm", "1_counter_collection.csv"), hdr, rows)
    out = P.valu_summary(raw, str(tmp_path / "v.md"), "cmd")
    single = out[0]
    assert single[6] == pytest.approx(2e8 * 4 / (1024 * 1e6))
    assert single[7] == pytest.approx(1e8 * 64 / P.N ** 2)
    batch = out[[p[0] for p in P.VALU_PASSES].index("batch512")]
    assert batch[2] == pytest.approx(2e8) and batch[7] == pytest.approx(2e8 * 64 / P.BATCH_NODES)
    d3 = out[[p[0] for p in P.VALU_PASSES].index("d3_f32")]
    assert d3[7] == pytest.approx(1e8 * 64 / P.N3 ** 3)
    assert "VALU busy" in open(tmp_path / "v.md").read()
    js = json.load(open(tmp_path / "v.json"))
    assert js["d3_f32"]["insts_per_node"] == pytest.approx(1e8 * 64 / P.N3 ** 3)
    assert js["d3_f32"]["kernel_source_sha"] == P.sources_sha(P.D3_SOURCES)
