"""Tile-shape tuning: fdlbm_autotune / fdlbm_batch_autotune pick a shape among their
candidates, leave the state untouched, and the tuned runs give the same bits as untuned
ones (the shape changes the speed only)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


@pytest.mark.parametrize("kw", [
    dict(scheme="fd", stencil=3, dtype="f32"),
    dict(scheme="fd", stencil=5, dtype="f64", bc="walls", force=(2e-5, -1e-5)),
    dict(scheme="fd", stencil=3, dtype="f16"),
    dict(scheme="mrt", dtype="f32", quartic=True),
    dict(scheme="fd", stencil=3, dtype="f32", kernel="reference"),
])
def test_autotune_keeps_state_and_results(F, kw):
    nx, ny = 520, 300
    print(f"case autotune {kw}", flush=True)
    r, x, y = W.random_state(nx, ny, seed=77, amp=0.02)
    out = []
    for tune in (False, True):
        sim = F.FdLbm(nx, ny, s_xx=1.6, s_e=1.1, **kw)
        sim.set_state(r, x, y)
        before = sim.get_state()
        if tune:
            cols, rows, ms = sim.autotune(reps=3)
            print(f"  chosen lane_cols={cols} tile_rows={rows} {ms:.4f} ms/step")
            assert ms > 0
            if kw.get("kernel") == "reference":
                assert (cols, rows) == (0, 0)
            elif kw["scheme"] == "fd":
                assert cols in (1, 2, 4) and rows in (4, 6, 8, 12, 16, 24)
            else:
                assert rows in (1, 2, 4, 8, 16)
            after = sim.get_state()
            assert sim.steps == 0
            for u, v in zip(before, after):
                assert np.array_equal(u, v)
        sim.step(15)
        out.append(sim.get_state())
        sim.close()
    for u, v in zip(*out):
        assert np.array_equal(u, v)


SPECS = [(33, 40, 1.6, 1.0), (64, 64, 1.2, 1.1), (100, 37, 1.85, 1.0), (8, 8, 1.5, 1.0), (250, 130, 1.9, 1.0)]


def test_batch_autotune_keeps_results(F):
    runs = []
    for tune in (False, True):
        b = F.FdLbmBatch(SPECS, dtype="f32", max_samples=4)
        for i, (nx, ny, _, _) in enumerate(SPECS):
            b.set_state(i, *W.random_state(nx, ny, seed=300 + i, amp=0.02))
        if tune:
            b.step(10, sample_every=5, use_graph=True)  # a cached replay that tuning must drop
            rows, ms = b.autotune(reps=2)
            print(f"  batch rows={rows} {ms:.4f} ms/step")
            assert rows in (4, 6, 8, 12, 16) and ms > 0
            assert b.steps == 10
            b.step(10, sample_every=5, use_graph=True)
        else:
            b.step(20, sample_every=5, use_graph=True)
        runs.append(([b.get_state(i) for i in range(len(SPECS))], b.amplitudes()))
        b.close()
    for sa, sb in zip(runs[0][0], runs[1][0]):
        for u, v in zip(sa, sb):
            assert np.array_equal(u, v)
    assert np.array_equal(runs[0][1], runs[1][1])
