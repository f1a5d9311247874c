"""The D3Q19 FD-LBM step on the GPU against the FP64 oracle, and the sweep kernel against the
reference kernels bit for bit.

Both GPU paths evaluate the same per-node arithmetic in the same order, so any difference
between them is a data-movement error (a lane shift, a row exchanged through LDS, a plane of
the register window, a wrap).  Shapes cover exact tiles, ragged strips, row bands and plane
bands (shifted back to the edge), grids smaller than one tile in every direction, and both
block heights.  At the benchmark size the step is checked on sampled nodes: one step at a node
depends only on the inputs within two nodes of it, so the oracle run on a periodic 9^3 window
around the node gives its exact new value.
"""
import numpy as np
import pytest

import workloads as W
from oracle import d3q19 as D

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


def run3(F, shape, steps, init, **kw):
    nz, ny, nx = shape
    sim = F.FdLbm3D(nx, ny, nz, **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_state()
    sim.close()
    return out


def rel(a, b):
    num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b))
    den = sum(float(np.sum(y ** 2)) for y in b)
    return (num / den) ** 0.5


SHAPES = [(32, 14, 60), (37, 19, 67), (3, 3, 3), (4, 5, 7), (9, 30, 130), (70, 12, 61)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_reference_matches_oracle(F, dtype, shape):
    print(f"case d3 reference-vs-oracle dtype={dtype} shape={shape}", flush=True)
    init = W.random_state3(shape[2], shape[1], shape[0], seed=sum(shape), amp=0.02)
    got = run3(F, shape, 6, init, dtype=dtype, s_nu=1.6, s_e=1.2, kernel="reference")
    want = D.fd3d_run(*init, 6, s_nu=1.6, s_e=1.2)
    assert rel(got, want) < (1e-13 if dtype == "f64" else 2e-6), rel(got, want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tile", [(0, 0), (8, 5), (12, 3), (16, 1), (8, 64)])
def test_sweep_equals_reference_bitwise(F, dtype, shape, tile):
    rows, planes = tile
    print(f"case d3 sweep-vs-reference dtype={dtype} shape={shape} tile_rows={rows} tile_planes={planes}",
          flush=True)
    init = W.random_state3(shape[2], shape[1], shape[0], seed=7 * sum(shape), amp=0.02)
    kw = dict(dtype=dtype, s_nu=1.45, s_e=1.15)
    a = run3(F, shape, 5, init, kernel="reference", **kw)
    b = run3(F, shape, 5, init, kernel="sweep", tile_rows=rows, tile_planes=planes, **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_sweep_matches_oracle_in_a_mean_flow(F):
    """Every nonlinear term of the defects acts: a random state on a uniform flow, s_e != 1."""
    shape = (20, 17, 64)
    print(f"case d3 sweep-vs-oracle mean flow shape={shape}", flush=True)
    r = W.random_state3(shape[2], shape[1], shape[0], seed=31, amp=0.01)
    init = (r[0], r[1] + 0.05, r[2] - 0.03, r[3] + 0.04)
    got = run3(F, shape, 20, init, dtype="f64", s_nu=1.7, s_e=1.4)
    want = D.fd3d_run(*init, 20, s_nu=1.7, s_e=1.4)
    assert rel(got, want) < 1e-13, rel(got, want)
    got32 = run3(F, shape, 20, init, dtype="f32", s_nu=1.7, s_e=1.4)
    assert rel(got32, want) < 1e-6, rel(got32, want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_conservation_and_diagnostics(F, dtype):
    shape = (24, 28, 90)
    print(f"case d3 conservation dtype={dtype} shape={shape}", flush=True)
    nz, ny, nx = shape
    init = W.random_state3(nx, ny, nz, seed=3, amp=0.02)
    sim = F.FdLbm3D(nx, ny, nz, dtype=dtype, s_nu=1.8, s_e=1.3)
    sim.set_state(*init)
    d0 = sim.diagnostics()
    want0 = [float(np.sum(a)) for a in init]
    if dtype == "f64":
        assert abs(d0["mass"] - want0[0]) < 1e-12 and abs(d0["mom_z"] - want0[3]) < 1e-12
    sim.step(200)
    d1 = sim.diagnostics()
    sim.close()
    tol = 1e-12 if dtype == "f64" else 2e-3
    for k in ("mass", "mom_x", "mom_y", "mom_z"):
        assert abs(d1[k] - d0[k]) < tol, (k, d0[k], d1[k])
    assert d1["nonfinite"] == 0 and d1["kin_energy"] < d0["kin_energy"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_shear_wave_decays_at_the_symbol_rate(F, dtype):
    """A transverse wave along the body diagonal of a 48^3 grid decays at the rate of the
    symbol's shear root (the amplitude is small enough that the nonlinear terms are below the
    tolerance)."""
    n, m, s_nu = 48, (1, 1, 1), 1.5
    print(f"case d3 shear wave dtype={dtype} n={n}", flush=True)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ph = 2 * np.pi * (x + y + z) / n
    amp = 1e-4
    jx, jy = amp * np.sin(ph), -amp * np.sin(ph)  # J perpendicular to k = (1, 1, 1)
    zero = np.zeros_like(jx)
    sim = F.FdLbm3D(n, n, n, dtype=dtype, s_nu=s_nu, s_e=1.2)
    sim.set_state(zero, jx, jy, zero)
    sim.step(400)
    out = sim.get_state()
    sim.close()
    k = 2 * np.pi * np.array(m) / n
    g = -np.log(np.linalg.eigvals(D.fd3d_symbol(k, s_nu=s_nu, s_e=1.2)))
    shear = g[np.argsort(np.abs(g.imag))[0]].real
    got = np.sum(out[1] * np.sin(ph)) / np.sum(np.sin(ph) ** 2)
    want = amp * np.exp(-400 * shear)
    assert abs(got / want - 1) < (1e-6 if dtype == "f64" else 1e-4), (got, want)


def sampled_one_step(F, shape, dtype, nsamples, seed, **kw):
    """One GPU step of the band-limited flow; returns the worst relative error over sampled
    nodes against the oracle run on the 9^3 periodic window around each node."""
    nz, ny, nx = shape
    init = W.decaying_flow3(nx, seed=seed, amp=0.02) if nx == ny == nz else None
    assert init is not None
    if dtype == "f32":
        init = tuple(a.astype(np.float32).astype(np.float64) for a in init)  # the values the GPU holds
    sim = F.FdLbm3D(nx, ny, nz, dtype=dtype, **kw)
    sim.set_state(*init)
    sim.step(1)
    out = sim.get_state()
    sim.close()
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, [nz, ny, nx], size=(nsamples, 3))
    pts[0] = (0, 0, 0)
    pts[1] = (nz - 1, ny - 1, nx - 1)
    worst = 0.0
    scale = max(float(np.max(np.abs(a))) for a in init)
    for (k, j, i) in pts:
        idx = np.ix_(np.arange(k - 4, k + 5) % nz, np.arange(j - 4, j + 5) % ny, np.arange(i - 4, i + 5) % nx)
        win = [a[idx] for a in init]
        res = D.fd3d_run(*win, 1, s_nu=kw["s_nu"], s_e=kw["s_e"])
        for q in range(4):
            worst = max(worst, abs(res[q][4, 4, 4] - out[q][k, j, i]) / scale)
    return worst


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_full_size_sampled_nodes_match_oracle(F, dtype):
    """At the 512^3 size of the measurement (the launch shape the bench times), 300 sampled
    nodes (two of them grid corners) of one step equal the oracle's: to 1e-6 of the field scale
    in FP32 (the roundings of one step), 1e-14 in FP64."""
    n = 512
    print(f"case d3 full-size sampled dtype={dtype} n={n}", flush=True)
    worst = sampled_one_step(F, (n, n, n), dtype, 300, seed=9, s_nu=1.0 / (0.5 + 3 * 0.02), s_e=1.0)
    assert worst < (1e-6 if dtype == "f32" else 1e-14), worst


def test_full_size_sweep_equals_reference(F):
    """At 512^3 the sweep kernel (the bench's launch shape) and the reference kernels give the
    same bits after three steps."""
    n = 512
    print(f"case d3 full-size sweep-vs-reference n={n}", flush=True)
    init = W.decaying_flow3(n, seed=9, amp=0.02)
    kw = dict(dtype="f32", s_nu=1.0 / (0.5 + 3 * 0.02), s_e=1.0)
    a = run3(F, (n, n, n), 3, init, kernel="reference", **kw)
    b = run3(F, (n, n, n), 3, init, kernel="sweep", **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_autotune_keeps_the_state_and_the_bits(F):
    """fdlbm3d_autotune times every tile shape out of place: the state and the step count are
    unchanged, and the tuned run gives the same bits as an untuned one."""
    shape = (40, 37, 130)
    print(f"case d3 autotune shape={shape}", flush=True)
    nz, ny, nx = shape
    init = W.random_state3(nx, ny, nz, seed=21, amp=0.02)
    sim = F.FdLbm3D(nx, ny, nz, dtype="f32", s_nu=1.5, s_e=1.1)
    sim.set_state(*init)
    before = sim.get_state()
    rows, planes, ms = sim.autotune(reps=2)
    assert rows in (8, 12, 16) and planes in (16, 32, 64, 128) and ms > 0
    assert sim.steps == 0
    for u, v in zip(before, sim.get_state()):
        assert np.array_equal(u, v)
    sim.step(7)
    tuned = sim.get_state()
    sim.close()
    plain = run3(F, shape, 7, init, dtype="f32", s_nu=1.5, s_e=1.1)
    for u, v in zip(tuned, plain):
        assert np.array_equal(u, v)


def test_fp32_long_run_against_fp64(F):
    """Over 1000 steps of the 128^3 decaying flow the FP32 state stays within 2e-6 (relative
    L2) of the FP64 run, whose kernels equal the oracle to 1e-13 above: the increment-form
    update keeps the rounding at the scale of the increments."""
    n, steps = 128, 1000
    print(f"case d3 fp32-vs-fp64 n={n} steps={steps}", flush=True)
    init = W.decaying_flow3(n, seed=6, amp=0.02)
    kw = dict(s_nu=1.0 / (0.5 + 3 * 0.02), s_e=1.0)
    a = run3(F, (n, n, n), steps, init, dtype="f64", **kw)
    b = run3(F, (n, n, n), steps, init, dtype="f32", **kw)
    err = rel(b, a)
    print(f"d3 fp32 vs fp64 after {steps} steps: {err:.3e}", flush=True)
    assert err < 2e-6, err


def test_state_beyond_2_31_values(F):
    """832 x 832 x 800 nodes: the four planes hold 2.2e9 values, more than 2^31, so every offset
    past the first plane needs 64-bit arithmetic.  A transverse wave along z plus a density wave
    along x; one step is checked on sampled nodes against the oracle (periodic 9^3 windows), and
    the FP64 momentum sums are conserved."""
    nx, ny, nz = 832, 832, 800
    print(f"case d3 beyond 2^31 values shape=({nz}, {ny}, {nx})", flush=True)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    shape = (nz, ny, nx)
    dr = np.ascontiguousarray(np.broadcast_to(1e-3 * np.cos(2 * np.pi * x / nx), shape))
    jx = np.ascontiguousarray(np.broadcast_to(2e-3 * np.sin(2 * np.pi * z / nz), shape))
    jy = np.zeros(shape)
    jz = np.ascontiguousarray(np.broadcast_to(1e-3 * np.cos(4 * np.pi * z / nz), shape))
    init = (dr, jx, jy, jz)
    kw = dict(s_nu=1.0 / (0.5 + 3 * 0.02), s_e=1.3)
    sim = F.FdLbm3D(nx, ny, nz, dtype="f32", **kw)
    sim.set_state(*init)
    d0 = sim.diagnostics()
    sim.step(1)
    d1 = sim.diagnostics()
    out = sim.get_state()
    sim.close()
    held = tuple(a.astype(np.float32).astype(np.float64) for a in init)
    rng = np.random.default_rng(3)
    pts = rng.integers(0, [nz, ny, nx], size=(60, 3))
    pts[0] = (nz - 1, ny - 1, nx - 1)
    worst = 0.0
    for (k, j, i) in pts:
        idx = np.ix_(np.arange(k - 4, k + 5) % nz, np.arange(j - 4, j + 5) % ny, np.arange(i - 4, i + 5) % nx)
        res = D.fd3d_run(*(a[idx] for a in held), 1, **kw)
        for q in range(4):
            worst = max(worst, abs(res[q][4, 4, 4] - out[q][k, j, i]) / 2e-3)
    assert worst < 1e-6, worst
    for key in ("mom_x", "mom_z"):
        assert abs(d1[key] - d0[key]) < 1e-6 * nx * ny * nz * 1e-3, (key, d0[key], d1[key])
    assert d1["nonfinite"] == 0
