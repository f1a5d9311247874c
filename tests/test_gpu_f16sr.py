"""FP16-stored deviations with stochastic rounding (FDLBM_F16DEV_SR) on the GPU: the sweep
kernels equal the reference kernels bit for bit (both draw the same counter-based bits), a
run is reproducible, and unbiased rounding keeps the increments that rounding to nearest
loses: a slow shear wave that stays frozen in FP16 decays at the dispersion rate, and mass
and momentum are conserved up to a random walk (full-size check in test_gpu_workloads.py);
node by node it is not more accurate than rounding to nearest.
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


def run(F, init, steps, **kw):
    ny, nx = init[0].shape
    sim = F.FdLbm(nx, ny, **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("shape,tile_rows,lane_cols", [((296, 77), 0, 0), ((70, 46), 3, 2), ((523, 40), 5, 4),
                                                       ((27, 9), 2, 1), ((250, 64), 16, 0)])
@pytest.mark.parametrize("case", ["fd3", "fd5", "fd3_force", "fd5_walls", "lwacm"])
def test_f16sr_sweep_equals_reference_bitwise(F, shape, tile_rows, lane_cols, case):
    nx, ny = shape
    if case.startswith("fd5") and lane_cols == 1:
        pytest.skip("5-point differences need two columns per lane")
    print(f"case f16sr sweep-vs-reference {case} shape={shape} tile_rows={tile_rows} lane_cols={lane_cols}",
          flush=True)
    init = W.random_state(nx, ny, seed=nx + ny, amp=0.02)
    kw = dict(dtype="f16sr", s_xx=O.rate_from_viscosity(0.03))
    if case == "lwacm":
        kw["scheme"] = "lwacm"
    else:
        kw.update(scheme="fd", stencil=int(case[2]), s_e=1.1)
        if case.endswith("force"):
            kw["force"] = (3e-6, -2e-6)
        if case.endswith("walls"):
            kw.update(bc="walls", wall_xi=0.3)
    a = run(F, init, 30, kernel="reference", **kw)
    b = run(F, init, 30, kernel="sweep", tile_rows=tile_rows, lane_cols=lane_cols, **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v), float(np.max(np.abs(u - v)))


def test_f16sr_is_reproducible_and_differs_from_rounding_to_nearest(F):
    init = W.random_state(96, 64, seed=5, amp=0.02)
    kw = dict(stencil=3, s_xx=O.rate_from_viscosity(0.02))
    a = run(F, init, 50, dtype="f16sr", **kw)
    b = run(F, init, 50, dtype="f16sr", **kw)
    c = run(F, init, 50, dtype="f16", **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert any(not np.array_equal(u, v) for u, v in zip(a, c))
    want = O.fd_run(*init, 50, s_xx=O.rate_from_viscosity(0.02), stencil=3)
    assert rel_l2(a, want) < 2e-3


def test_f16sr_slow_shear_wave_decays_at_the_dispersion_rate(F):
    """jx = 0.01 sin(2 pi y / 512), nu = 0.01: each step removes about 1.5e-8 from a value
    whose FP16 unit is 7.6e-6, so rounding to nearest returns every node to its old value and
    the wave never decays.  With stochastic rounding A(t) follows exp(-Gamma t), Gamma the
    shear root of the amplification matrix, over 20 000 steps."""
    n, nu, steps = 512, 0.01, 20000
    s_xx = O.rate_from_viscosity(nu)
    init = W.shear_wave_y(n, n, 0.01, 1)
    g = S.shear_gamma(0.0, 2 * math.pi / n, s_xx=s_xx, stencil=3).real
    want = math.exp(-g * steps)
    amps = {}
    for dtype in ("f16", "f16sr", "f32"):
        sim = F.FdLbm(n, n, dtype=dtype, stencil=3, s_xx=s_xx)
        sim.set_state(*init)
        sim.set_mode(init[1], init[2])
        a0 = sim.mode_projection()
        sim.step(steps)
        amps[dtype] = sim.mode_projection() / a0
        sim.close()
    print(f"  A({steps}): exp(-Gamma t) {want:.5f}, f32 {amps['f32']:.5f}, f16 {amps['f16']:.5f}, "
          f"f16sr {amps['f16sr']:.5f}")
    assert abs(amps["f32"] - want) < 2e-4
    assert abs(amps["f16sr"] - want) < 2e-3
    assert abs(amps["f16"] - want) > 1e-2  # rounding to nearest stalls the decay


def band_error(got, want, kmax=8):
    """Relative error of the Fourier modes 0 < |k| <= kmax (the band the input holds)."""
    num = den = 0.0
    for g, w in zip(got, want):
        n = w.shape[0]
        k = np.fft.fftfreq(n, 1.0 / n)
        band = (k[:, None] ** 2 + k[None, :] ** 2 <= kmax * kmax) & (k[:, None] ** 2 + k[None, :] ** 2 > 0)
        fg, fw = np.fft.fft2(g), np.fft.fft2(w)
        num += float(np.sum(np.abs(fg - fw)[band] ** 2))
        den += float(np.sum(np.abs(fw)[band] ** 2))
    return math.sqrt(num / den)


def test_f16sr_stokes_modes_256_against_the_oracle(F):
    """256^2 band-limited modes, 2000 steps, against the FP64 oracle.  Stochastic rounding is
    unbiased but not more accurate node by node: its per-node roundings add a small-scale
    random walk, so its relative L2 error is a little above that of rounding to nearest (both
    stay below 2e-3); its gain is in the slow, large-scale content (the shear-wave and
    conservation tests)."""
    init = W.stokes_modes_256(seed=3, rms=1e-2)
    steps = 2000
    for nu in (0.02, 0.005):
        s_xx = O.rate_from_viscosity(nu)
        want = O.fd_run(*init, steps, s_xx=s_xx, stencil=3)
        errs, bands = {}, {}
        for d in ("f16", "f16sr"):
            got = run(F, init, steps, dtype=d, stencil=3, s_xx=s_xx)
            errs[d], bands[d] = rel_l2(got, want), band_error(got, want)
        print(f"  256^2 nu={nu} {steps} steps: rel L2 f16 {errs['f16']:.2e}, f16sr {errs['f16sr']:.2e}; "
              f"in-band f16 {bands['f16']:.2e}, f16sr {bands['f16sr']:.2e}")
        assert errs["f16"] < 2e-3 and errs["f16sr"] < 2e-3


@pytest.mark.parametrize("case", ["fd3", "fd5_walls", "lwacm"])
def test_restore_mid_run_continues_bit_for_bit(F, case):
    """A run saved at step k (fdlbm_get_state plus fdlbm_step_count) and restored in a new
    context (fdlbm_set_state plus fdlbm_set_step_count) continues with the same random bits:
    its next steps equal those of the uninterrupted run bit for bit.  Restoring the state
    alone restarts the count at 0 and replays the first steps' bits instead."""
    nx, ny, k, more = 130, 41, 7, 9
    print(f"case f16sr restore {case} k={k}", flush=True)
    kw = dict(dtype="f16sr", s_xx=O.rate_from_viscosity(0.02))
    if case == "lwacm":
        kw["scheme"] = "lwacm"
    else:
        kw.update(scheme="fd", stencil=int(case[2]), s_e=1.1)
        if case.endswith("walls"):
            kw.update(bc="walls", force=(1e-5, 0.0))
    init = W.random_state(nx, ny, seed=11, amp=0.02)
    a = F.FdLbm(nx, ny, **kw)
    a.set_state(*init)
    a.step(k)
    saved, count = a.get_state(), a.steps
    a.step(more)
    want = a.get_state()
    a.close()
    assert count == k
    b = F.FdLbm(nx, ny, **kw)
    b.set_state(*saved)
    assert b.steps == 0
    b.steps = count
    b.step(more)
    got = b.get_state()
    assert b.steps == k + more
    # without the count: the first steps' bits, a different rounding
    b.set_state(*saved)
    b.step(more)
    replay = b.get_state()
    b.close()
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert any(not np.array_equal(r, w) for r, w in zip(replay, want))
