"""Walls at a general distance xi beyond the first and last rows (sections 3-b, 3-c, Fig. 6)
on the GPU: the FD-LBM sweep kernel bit for bit against the reference kernel, FD-LBM and
MRT (interpolated bounce-back) against the FP64 oracle, and the wall location measured
from the steady channel profile against the oracle's.
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


def rel_l2(a, b):
    return math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b)) / sum(float(np.sum(y * y)) for y in b))


def run(F, init, steps, **kw):
    ny, nx = init[0].shape
    sim = F.FdLbm(nx, ny, bc="walls", **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("xi", [0.2, 0.7, 1.0])
@pytest.mark.parametrize("shape,tile_rows", [((296, 77), 0), ((24, 9), 2), ((523, 40), 3)])
@pytest.mark.parametrize("forced", [False, True])
def test_sweep_general_xi_equals_reference_bitwise(F, dtype, stencil, xi, shape, tile_rows, forced):
    nx, ny = shape
    print(f"case walls xi={xi} dtype={dtype} stencil={stencil} shape={shape} tile_rows={tile_rows} forced={forced}",
          flush=True)
    init = W.random_state(nx, ny, seed=nx + 7 * ny, amp=0.02)
    kw = dict(scheme="fd", stencil=stencil, dtype=dtype, s_xx=1.6, s_e=1.1, wall_xi=xi,
              force=(2e-5, -1e-5) if forced else (0.0, 0.0))
    a = run(F, init, 9, kernel="reference", **kw)
    b = run(F, init, 9, kernel="sweep", tile_rows=tile_rows, **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v), float(np.max(np.abs(u - v)))


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("xi", [0.3, 0.8])
def test_general_xi_matches_oracle(F, scheme, dtype, tol, xi):
    nx, ny, steps, fx = 48, 37, 60, 1e-5
    init = W.random_state(nx, ny, seed=41, amp=0.02)
    s_xx = 1.6
    if scheme == "mrt":
        got = run(F, init, steps, scheme="mrt", dtype=dtype, s_xx=s_xx, quartic=True, wall_xi=xi, force=(fx, 0.0))
        want = O.mrt_moments(O.mrt_run(O.mrt_init(*init), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx), walls=True,
                                       xi=xi, fx=fx))
    else:
        st = int(scheme[2])
        got = run(F, init, steps, scheme="fd", stencil=st, dtype=dtype, s_xx=s_xx, s_e=1.0, wall_xi=xi,
                  force=(fx, 0.0))
        want = O.fd_run(*init, steps, s_xx=s_xx, s_e=1.0, stencil=st, walls=True, xi=xi, fx=fx)
    err = rel_l2(got, want)
    print(f"  walls xi={xi} {scheme} {dtype}: rel L2 {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_channel_wall_location_fig6(F, scheme):
    """Channel [1 - xi, 15 + xi] driven by a body force (nu = 1/sqrt(108)), FP64, 4000 steps
    from the analytic parabola: the zero of the fitted steady profile equals the oracle's
    to 1e-9 and follows the imposed xi."""
    nx, ny, nu, uc, steps = 8, 15, 1 / math.sqrt(108), 0.01, 4000
    s_xx = O.rate_from_viscosity(nu)
    y = np.arange(ny, dtype=float)
    for xi in (0.25, 0.5, 0.75, 1.0):
        L = ny - 1 + 2 * xi
        fx = 8 * nu * uc / L ** 2
        u = fx / (2 * nu) * (y + xi) * (ny - 1 + xi - y)
        init = (np.zeros((ny, nx)), np.repeat(u[:, None], nx, 1) - fx / 2, np.zeros((ny, nx)))
        if scheme == "mrt":
            got = run(F, init, steps, scheme="mrt", dtype="f64", s_xx=s_xx, quartic=True, wall_xi=xi,
                      force=(fx, 0.0))
            want = O.mrt_moments(O.mrt_run(O.mrt_init(*init), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx), walls=True,
                                           xi=xi, fx=fx))
        else:
            st = int(scheme[2])
            got = run(F, init, steps, scheme="fd", stencil=st, dtype="f64", s_xx=s_xx, s_e=1.0, wall_xi=xi,
                      force=(fx, 0.0))
            want = O.fd_run(*init, steps, s_xx=s_xx, s_e=1.0, stencil=st, walls=True, xi=xi, fx=fx)
        zeros = []
        for state in (got, want):
            prof = state[1][:, 0] + fx / 2
            lo, hi = np.sort(np.roots(np.polyfit(y, prof, 2)).real)
            zeros.append(-lo)
            assert abs(-lo - (hi - (ny - 1))) < 1e-9
        print(f"  {scheme} xi={xi}: measured {zeros[0]:.4f} (oracle {zeros[1]:.4f})")
        assert abs(zeros[0] - zeros[1]) < 1e-9
        assert abs(zeros[0] - xi) < 0.06


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
@pytest.mark.parametrize("xi", [0.5, 0.2, 1.0])
def test_narrowest_channel(F, scheme, xi):
    """The smallest channel the ABI accepts, 4 rows between the walls (every fluid row is then
    within reach of a wall and the ghost rows of both walls meet): FD-LBM sweep equals the
    reference kernel bit for bit, and FP64 and FP32 match the oracle after 50 steps."""
    nx, ny, steps, fx = 40, 4, 50, 1e-5
    print(f"case narrowest channel {scheme} xi={xi}", flush=True)
    init = W.random_state(nx, ny, seed=9, amp=0.02)
    if scheme == "mrt":
        want = O.mrt_moments(O.mrt_run(O.mrt_init(*init), steps, s_xx=1.6, s_q=O.quartic_s_q(1.6), walls=True, xi=xi,
                                       fx=fx))
        for dtype, tol in (("f64", 1e-12), ("f32", 1e-5)):
            got = run(F, init, steps, scheme="mrt", dtype=dtype, s_xx=1.6, quartic=True, wall_xi=xi, force=(fx, 0.0))
            assert rel_l2(got, want) <= tol, (dtype, rel_l2(got, want))
        return
    st = int(scheme[2])
    kw = dict(scheme="fd", stencil=st, s_xx=1.6, s_e=1.0, wall_xi=xi, force=(fx, 0.0))
    want = O.fd_run(*init, steps, s_xx=1.6, s_e=1.0, stencil=st, walls=True, xi=xi, fx=fx)
    for dtype, tol in (("f64", 1e-12), ("f32", 1e-5)):
        a = run(F, init, steps, kernel="reference", dtype=dtype, **kw)
        b = run(F, init, steps, kernel="sweep", dtype=dtype, **kw)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
        err = rel_l2(b, want)
        print(f"  {scheme} {dtype} xi={xi}: rel L2 {err:.2e}")
        assert err <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("xi", [0.2, 0.35, 0.5, 0.8, 1.0])
@pytest.mark.parametrize("shape,tile_rows", [((296, 77), 0), ((70, 9), 2), ((523, 40), 3), ((41, 4), 16)])
@pytest.mark.parametrize("forced", [False, True])
def test_mrt_sweep_general_xi_equals_reference_bitwise(F, dtype, xi, shape, tile_rows, forced):
    """The MRT vector sweep applies the interpolated bounce-back itself (for xi < 1/2 it
    collides the row next to the wall once more and takes f*_k(x - e_k) across lanes):
    populations equal the one-thread-per-node kernel's bit for bit, at every lane width
    (nx a multiple of 4, even, odd), tile height and the 4-row channel."""
    nx, ny = shape
    print(f"case mrt walls xi={xi} dtype={dtype} shape={shape} tile_rows={tile_rows} forced={forced}", flush=True)
    init = W.random_state(nx, ny, seed=nx + 3 * ny, amp=0.02)
    kw = dict(scheme="mrt", dtype=dtype, s_xx=1.6, s_e=1.1, s_q=1.2, s_eps=1.3, wall_xi=xi,
              force=(2e-5, -1e-5) if forced else (0.0, 0.0))
    out = []
    for kernel, rows in (("reference", 0), ("sweep", tile_rows)):
        sim = F.FdLbm(nx, ny, bc="walls", kernel=kernel, tile_rows=rows, **kw)
        sim.set_state(*init)
        sim.step(9)
        out.append(sim.get_populations())
        sim.close()
    assert np.array_equal(out[0], out[1]), float(np.max(np.abs(out[0] - out[1])))
