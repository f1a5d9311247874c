"""The LW-ACM step (section 1-b) on the GPU: the sweep kernel bit for bit against the
reference kernel, both against the FP64 oracle, and the Galilean test of section 3-a
(Fig. 1): the correlation A(t) of a transverse wave in a mean flow V, sampled by the
library's FP64 device projection, against the oracle's amplification matrix.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import symbol as S

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


def run(F, kernel, init, steps, **kw):
    ny, nx = init[0].shape
    sim = F.FdLbm(nx, ny, scheme="lwacm", kernel=kernel, **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("shape,tile_rows", [((296, 77), 0), ((9, 13), 5), ((523, 40), 3), ((250, 64), 16),
                                              ((27, 9), 2)])
@pytest.mark.parametrize("lane_cols", [1, 2, 4])
def test_lwacm_sweep_equals_reference_bitwise(F, dtype, shape, tile_rows, lane_cols):
    """Every lane width and access mode (aligned, element-aligned, per column) and ragged
    strips and bands give the reference kernel's bits."""
    if lane_cols == 4 and dtype == "f64":
        pytest.skip("FP64 takes at most 2 columns per lane")
    nx, ny = shape
    print(f"case lwacm sweep-vs-reference dtype={dtype} shape={shape} tile_rows={tile_rows} lane_cols={lane_cols}",
          flush=True)
    init = W.random_state(nx, ny, seed=nx + 3 * ny, amp=0.02)
    kw = dict(dtype=dtype, s_xx=O.rate_from_viscosity(0.03))
    a = run(F, "reference", init, 9, **kw)
    b = run(F, "sweep", init, 9, tile_rows=tile_rows, lane_cols=lane_cols, **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v), float(np.max(np.abs(u - v)))


@pytest.mark.parametrize("kernel", ["reference", "sweep"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_lwacm_matches_oracle(F, kernel, dtype, tol):
    init = W.stokes_modes_256(seed=3, rms=1e-2)
    nu, steps = 0.05, 200
    got = run(F, kernel, init, steps, dtype=dtype, s_xx=O.rate_from_viscosity(nu))
    want = O.lwacm_run(*init, steps, nu=nu)
    err = rel_l2(got, want)
    print(f"  lwacm {kernel} {dtype} 256^2 200 steps rel L2 {err:.2e}")
    assert err <= tol


def test_lwacm_f16_storage_error(F):
    """FP16 storage with FP32 arithmetic: the storage rounding (2^-11 relative) bounds the
    error against the FP64 oracle; it does not grow over 400 steps."""
    n, nu = 128, 0.02
    state = W.decaying_flow(n=n, seed=4, kmax=16, amp=0.02)
    sim = F.FdLbm(n, n, scheme="lwacm", dtype="f16", s_xx=O.rate_from_viscosity(nu))
    sim.set_state(*state)
    errs = []
    for _ in range(4):
        sim.step(100)
        state = O.lwacm_run(*state, 100, nu=nu)
        errs.append(rel_l2(sim.get_state(), state))
    sim.close()
    print("  lwacm f16 rel L2 after 100..400 steps:", ["%.2e" % e for e in errs])
    assert max(errs) <= 5e-3
    assert errs[-1] <= 2.0 * errs[0] + 1e-4


def test_lwacm_full_size_band_against_oracle(F):
    """8192 x 8192 decaying flow, FP32, default launch: a 64-row band after 8 steps against
    the oracle run on that band plus its domain of dependence (8 rows each side)."""
    n, steps, nu = 8192, 8, 0.02
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    got = run(F, "auto", init, steps, dtype="f32", s_xx=O.rate_from_viscosity(nu))
    y0, h, pad = 4000, 64, steps + 2
    band = tuple(a[y0 - pad:y0 + h + pad].copy() for a in init)
    want = O.lwacm_run(*band, steps, nu=nu)
    err = rel_l2([g[y0:y0 + h] for g in got], [w[pad:pad + h] for w in want])
    print(f"  lwacm 8192^2 band rel L2 {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("V", [0.0, 0.05, 0.1, 0.15, 0.2])
def test_lwacm_galilean_correlation_fig1(F, V):
    """Section 3-a, Fig. 1: 191 x 191 periodic square, transverse wave of wave vector
    (3 k0, 2 k0), k0 = 2 pi / 191, mean flow V along it (nu = 0.05, c_s = 0.32).
    A(t) = <J(t), J0'> / <J0', J0'> with J0' the initial wave, sampled on the device every
    25 steps, equals Re[(H^t Phi0)_J . t] / a for the oracle's amplification matrix H
    (FP64, amplitude a = 1e-6, so the wave is linear about the flow).  The damping falls
    as V grows, as nu - V^2/2."""
    n, nu, a, mx, my = 191, 0.05, 1e-6, 3, 2
    r, jx, jy = W.shear_wave(n, n, a, mx, my, V=V)
    kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
    k = math.hypot(kx, ky)
    t = np.array([-ky / k, kx / k])
    vx, vy = V * kx / k, V * ky / k
    sim = F.FdLbm(n, n, scheme="lwacm", dtype="f64", s_xx=O.rate_from_viscosity(nu))
    sim.set_state(r, jx, jy)
    sim.set_mode(jx - vx, jy - vy)
    H = S.lwacm_symbol(kx, ky, nu=nu, vx=vx, vy=vy)
    phi = np.array([0.0, a * t[0], a * t[1]], dtype=complex)
    got, want = [], []
    for step in range(0, 1001, 25):
        got.append(sim.mode_projection())
        want.append(float(np.real(phi[1] * t[0] + phi[2] * t[1])) / a)
        sim.step(25)
        phi = np.linalg.matrix_power(H, 25) @ phi
    sim.close()
    got, want = np.array(got), np.array(want)
    print(f"  V={V}: A(1000) = {got[-1]:.6f} (matrix {want[-1]:.6f}), max |diff| {np.max(np.abs(got - want)):.1e}")
    assert np.max(np.abs(got - want)) < 1e-6
    gamma = -np.log(abs(np.linalg.eigvals(H)))
    shear = float(np.min(gamma))  # the slowest root is the shear one at this k
    assert abs(shear / k ** 2 - (nu - V * V / 2)) < 0.005 * nu, (shear / k ** 2, nu - V * V / 2)
