"""The fused sweep kernel against the reference kernel (bit for bit) and the oracle.

Both kernels evaluate the same per-node arithmetic in the same order, so any difference
is a data-movement error: a wrong lane shift, window slot, strip overlap, wrap, ghost row
or a partial sum exchanged between the stacked wavefronts of a block.  Shapes are chosen
so that strips are partial in x (widths that are not multiples of the strip width, nor of
the lane group), the grid can be narrower than one strip, row bands end early (with a single leftover row
absorbed by the wavefront below, or a band of one row), and the rows per wavefront vary
(including fewer than the row window).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


def run(F, kernel, nx, ny, steps, init, **kw):
    sim = F.FdLbm(nx, ny, kernel=kernel, **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape,tile_rows", [((296, 77), 0), ((8, 13), 5), ((520, 40), 3), ((252, 64), 16),
                                              ((24, 9), 2)])
@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("forced", [False, True])
def test_sweep_equals_reference_bitwise(F, dtype, stencil, walls, shape, tile_rows, wide, forced):
    nx, ny = shape
    lane_cols = {"f64": (2, 1), "f32": (2, 4), "f16": (2, 4)}[dtype][int(wide)]
    if lane_cols == 1 and stencil == 5:
        lane_cols = 2
    print(f"case sweep-vs-reference dtype={dtype} stencil={stencil} walls={walls} shape={shape} "
          f"tile_rows={tile_rows} lane_cols={lane_cols} forced={forced}", flush=True)
    init = W.random_state(nx, ny, seed=nx + ny, amp=0.02)
    kw = dict(stencil=stencil, dtype=dtype, bc="walls" if walls else "periodic", s_xx=1.6, s_e=1.1,
              force=(2e-5, -1e-5) if forced else (0.0, 0.0))
    a = run(F, "reference", nx, ny, 9, init, **kw)
    b = run(F, "sweep", nx, ny, 9, init, tile_rows=tile_rows, lane_cols=lane_cols, **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v), float(np.max(np.abs(u - v)))


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape,tile_rows", [((297, 77), 0), ((9, 13), 5), ((523, 40), 3), ((250, 64), 16),
                                              ((27, 9), 2)])
@pytest.mark.parametrize("narrow", [False, True])
@pytest.mark.parametrize("forced", [False, True])
def test_sweep_per_column_access_equals_reference_bitwise(F, dtype, stencil, walls, shape, tile_rows, narrow,
                                                          forced):
    """Widths that are not a multiple of the lane group (odd, or 2 mod 4): each column is
    loaded and stored on its own and wraps across the periodic edge on its own, at 4 (FP32,
    FP16) or 2 columns per lane; the 9-wide grid wraps many times inside one strip."""
    nx, ny = shape
    lane_cols = 2 if narrow or dtype == "f64" else 4
    if narrow and dtype == "f64":
        pytest.skip("FP64 has one lane width with 16-byte accesses")
    print(f"case per-column dtype={dtype} stencil={stencil} walls={walls} shape={shape} "
          f"tile_rows={tile_rows} lane_cols={lane_cols} forced={forced}", flush=True)
    init = W.random_state(nx, ny, seed=nx * ny, amp=0.02)
    kw = dict(stencil=stencil, dtype=dtype, bc="walls" if walls else "periodic", s_xx=1.6, s_e=1.1,
              force=(2e-5, -1e-5) if forced else (0.0, 0.0))
    a = run(F, "reference", nx, ny, 9, init, **kw)
    b = run(F, "sweep", nx, ny, 9, init, tile_rows=tile_rows, lane_cols=lane_cols, **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v), float(np.max(np.abs(u - v)))


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("stencil", [3, 5])
def test_sweep_matches_oracle(F, dtype, tol, stencil):
    nx, ny, steps = 264, 70, 40
    init = W.random_state(nx, ny, seed=5, amp=0.02)
    got = run(F, "auto", nx, ny, steps, init, stencil=stencil, dtype=dtype, s_xx=1.7, s_e=1.0)
    want = O.fd_run(*init, steps, s_xx=1.7, s_e=1.0, stencil=stencil)
    err = math.sqrt(sum(float(np.sum((g - w) ** 2)) for g, w in zip(got, want)) /
                    sum(float(np.sum(w * w)) for w in want))
    print(f"  sweep {dtype} FD{stencil} rel L2 {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f16", 5e-3)])
def test_full_size_band_against_oracle(F, dtype, tol):
    """8192 x 8192 decaying flow in the launch configuration the bench times: after 12
    steps, 256 rows are compared with the oracle run on those rows plus the 24-row domain of
    dependence on each side."""
    n, steps, rows, y0 = 8192, 12, 256, 3000
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    s_xx = O.rate_from_viscosity(0.02)
    got = run(F, "auto", n, n, steps, init, stencil=3, dtype=dtype, s_xx=s_xx, s_e=1.0)
    m = 2 * steps
    band = tuple(np.ascontiguousarray(a[y0 - m:y0 + rows + m]) for a in init)
    want = [a[m:m + rows] for a in O.fd_run(*band, steps, s_xx=s_xx, s_e=1.0, stencil=3)]
    err = math.sqrt(sum(float(np.sum((g[y0:y0 + rows] - w) ** 2)) for g, w in zip(got, want)) /
                    sum(float(np.sum(w * w)) for w in want))
    print(f"  8192^2 {dtype} band rel L2 {err:.2e}")
    assert err <= tol
