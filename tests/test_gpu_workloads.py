"""The configurations of the build at their own sizes, on the GPU.

* 256 x 256 "Stokes modes": band-limited random fields (modes 0 < |k| <= 8).  Against the
  oracle over 200 steps, and -- at tiny amplitude, where the scheme is linear -- every
  sampled Fourier mode after 2000 steps against the amplification matrix H(k)^2000
  (decay of the shear root, speed and damping of the sound roots).
* Poiseuille channel 16384 x 1024 with walls and a body force (section 3-c), FP32: the
  x-invariant profile against the FP64 oracle on an 8-column channel, and the analytic
  parabola.
* 8192 x 8192 decaying flow over 2000 steps: FP32 and FP16 storage against the FP64 GPU
  run (itself checked against the oracle at this size in test_gpu_sweep.py).
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


def fourier(f, mx, my):
    ny, nx = f.shape[-2:]
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.sum(f * np.exp(-2j * np.pi * (mx * x / nx + my * y / ny)), axis=(-2, -1))


def run_gpu(F, init, steps, **kw):
    ny, nx = init[0].shape
    sim = F.FdLbm(nx, ny, **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_populations() if kw.get("scheme") == "mrt" else sim.get_state()
    sim.close()
    return out


NU = 0.05  # Table 2's long-wavelength viscosity


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_stokes_modes_256_against_oracle(F, scheme, dtype, tol):
    init = W.stokes_modes_256(seed=2)
    s_xx = O.rate_from_viscosity(NU)
    steps = 200
    if scheme == "mrt":
        got = run_gpu(F, init, steps, scheme="mrt", dtype=dtype, s_xx=s_xx, quartic=True)
        want = O.mrt_run(O.mrt_init(*init), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx))
        err = math.sqrt(float(np.sum((got - want) ** 2)) / float(np.sum(want ** 2)))
    else:
        st = int(scheme[2])
        got = run_gpu(F, init, steps, scheme="fd", stencil=st, dtype=dtype, s_xx=s_xx, s_e=1.0)
        want = O.fd_run(*init, steps, s_xx=s_xx, s_e=1.0, stencil=st)
        err = rel_l2(got, want)
    print(f"  256^2 {scheme} {dtype} 200 steps rel L2 {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_stokes_modes_256_dispersion(F, scheme):
    """At RMS amplitude 1e-12 the 2000-step evolution of each Fourier mode is H(k)^2000
    applied to its initial amplitudes (shear decay, sound speed and sound damping).  The
    residual is the quadratic coupling between modes: it scales with the amplitude (about
    240 x rms on the FP64 oracle for this field), so 1e-8 leaves a margin of 40."""
    init = W.stokes_modes_256(seed=2, rms=1e-12)
    n, steps = 256, 2000
    s_xx = O.rate_from_viscosity(NU)
    modes = [(1, 0), (3, 4), (8, 0), (5, 5), (6, -3), (0, 7)]
    if scheme == "mrt":
        s_q = O.quartic_s_q(s_xx)
        f0 = O.mrt_init(*init)
        got = run_gpu(F, init, steps, scheme="mrt", dtype="f64", s_xx=s_xx, quartic=True)
    else:
        st = int(scheme[2])
        got = run_gpu(F, init, steps, scheme="fd", stencil=st, dtype="f64", s_xx=s_xx, s_e=1.0)
    for m in modes:
        kx, ky = 2 * math.pi * m[0] / n, 2 * math.pi * m[1] / n
        if scheme == "mrt":
            H = S.mrt_symbol(kx, ky, s_xx=s_xx, s_q=s_q)
            phi0, phi = fourier(f0, *m), fourier(got, *m)
        else:
            H = S.fd_symbol(kx, ky, s_xx=s_xx, s_e=1.0, stencil=int(scheme[2]))
            phi0 = np.array([fourier(a, *m) for a in init])
            phi = np.array([fourier(a, *m) for a in got])
        pred = np.linalg.matrix_power(H, steps) @ phi0
        err = np.max(np.abs(phi - pred)) / np.max(np.abs(pred))
        assert err < 1e-8, (m, err)


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_stokes_modes_256_dispersion_10000_steps(F, scheme):
    """The same linear check over the configuration's 10000 steps, on the long-lived modes
    (|k| <= 2*pi*sqrt(5)/256), FP64: each mode equals H(k)^10000 applied to its initial
    amplitudes to 1e-7."""
    init = W.stokes_modes_256(seed=2, rms=1e-12)
    n, steps = 256, 10000
    s_xx = O.rate_from_viscosity(NU)
    modes = [(1, 0), (0, 1), (1, 1), (2, 1), (-1, 2)]
    if scheme == "mrt":
        s_q = O.quartic_s_q(s_xx)
        f0 = O.mrt_init(*init)
        got = run_gpu(F, init, steps, scheme="mrt", dtype="f64", s_xx=s_xx, quartic=True)
    else:
        got = run_gpu(F, init, steps, scheme="fd", stencil=int(scheme[2]), dtype="f64", s_xx=s_xx, s_e=1.0)
    for m in modes:
        kx, ky = 2 * math.pi * m[0] / n, 2 * math.pi * m[1] / n
        if scheme == "mrt":
            H = S.mrt_symbol(kx, ky, s_xx=s_xx, s_q=s_q)
            phi0, phi = fourier(f0, *m), fourier(got, *m)
        else:
            H = S.fd_symbol(kx, ky, s_xx=s_xx, s_e=1.0, stencil=int(scheme[2]))
            phi0 = np.array([fourier(a, *m) for a in init])
            phi = np.array([fourier(a, *m) for a in got])
        pred = np.linalg.matrix_power(H, steps) @ phi0
        err = np.max(np.abs(phi - pred)) / np.max(np.abs(pred))
        assert err < 1e-7, (m, err)


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_stokes_modes_256_fp32_10000_steps_against_oracle(F, scheme):
    """The 256^2 Stokes-mode configuration in FP32 over its full 10000 steps (RMS 1e-3, the
    nonlinear regime), every node against the FP64 oracle at every 2000 steps (relative L2
    <= 1e-5), and the decay rate of each long-lived shear mode fitted from the FP32 run
    against the same fit of the oracle run (to 1e-4).  At this amplitude the slowest modes
    exchange energy with the others at a rate k|J| ~ 2.5e-5, as fast as they decay (3e-5),
    so their rates are not the linear ones; the FP32 dispersion test below compares with
    the amplification matrix in the linear regime."""
    init = W.stokes_modes_256(seed=2)
    n, chunk, nchunks = 256, 2000, 5
    s_xx = O.rate_from_viscosity(NU)
    s_q = O.quartic_s_q(s_xx)
    print(f"  256^2 FP32 10000 steps {scheme}", flush=True)
    if scheme == "mrt":
        sim = F.FdLbm(n, n, scheme="mrt", dtype="f32", s_xx=s_xx, quartic=True)
        ref = O.mrt_init(*init)
    else:
        sim = F.FdLbm(n, n, scheme="fd", stencil=int(scheme[2]), dtype="f32", s_xx=s_xx, s_e=1.0)
        ref = tuple(init)
    sim.set_state(*init)
    modes = [(1, 0), (0, 1), (1, 1), (2, 1), (-1, 2), (2, 2)]

    def shear(state, m):
        k = np.array(m, dtype=float) / math.hypot(*m)
        return fourier(-k[1] * state[1] + k[0] * state[2], *m)

    amps_gpu, amps_ref, errs = [[shear(init, m) for m in modes]], [[shear(init, m) for m in modes]], []
    for c in range(nchunks):
        sim.step(chunk)
        got = sim.get_state()
        if scheme == "mrt":
            ref = O.mrt_run(ref, chunk, s_xx=s_xx, s_q=s_q)
            want = O.mrt_moments(ref)
        else:
            ref = O.fd_run(*ref, chunk, s_xx=s_xx, s_e=1.0, stencil=int(scheme[2]))
            want = ref
        errs.append(rel_l2(got, want))
        amps_gpu.append([shear(got, m) for m in modes])
        amps_ref.append([shear(want, m) for m in modes])
        print(f"    step {(c + 1) * chunk}: rel L2 {errs[-1]:.2e}", flush=True)
    sim.close()
    assert max(errs) <= 1e-5, errs
    t = np.arange(nchunks + 1) * chunk
    for j, m in enumerate(modes):
        kx, ky = 2 * math.pi * m[0] / n, 2 * math.pi * m[1] / n
        kw = dict(s_q=s_q) if scheme == "mrt" else dict(stencil=int(scheme[2]), s_e=1.0)
        g_sym = S.shear_gamma(kx, ky, "mrt" if scheme == "mrt" else "fd", s_xx=s_xx, **kw).real
        g_gpu = -np.polyfit(t, np.log(np.abs([a[j] for a in amps_gpu])), 1)[0]
        g_ref = -np.polyfit(t, np.log(np.abs([a[j] for a in amps_ref])), 1)[0]
        print(f"    mode {m}: Gamma FP32 {g_gpu:.6e} oracle {g_ref:.6e} (linear symbol {g_sym:.6e})")
        assert abs(g_gpu / g_ref - 1) < 1e-4, (m, g_gpu, g_ref)


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_stokes_modes_256_fp32_dispersion_10000_steps(F, scheme):
    """The linear check of the 10000-step FP64 test in FP32 storage and arithmetic, at RMS
    1e-6 (linear regime; the stored deviations keep full relative precision at any
    amplitude): every long-lived mode, shear and acoustic, equals H(k)^10000 applied to its
    initial amplitudes.  The FP32 residue is the random walk of per-step roundings: 3.8e-5
    measured for the three schemes, bounded here at 2e-4."""
    init = W.stokes_modes_256(seed=2, rms=1e-6)
    n, steps = 256, 10000
    s_xx = O.rate_from_viscosity(NU)
    modes = [(1, 0), (0, 1), (1, 1), (2, 1), (-1, 2)]
    if scheme == "mrt":
        s_q = O.quartic_s_q(s_xx)
        f0 = O.mrt_init(*init)
        got = run_gpu(F, init, steps, scheme="mrt", dtype="f32", s_xx=s_xx, quartic=True)
    else:
        got = run_gpu(F, init, steps, scheme="fd", stencil=int(scheme[2]), dtype="f32", s_xx=s_xx, s_e=1.0)
    worst = 0.0
    for m in modes:
        kx, ky = 2 * math.pi * m[0] / n, 2 * math.pi * m[1] / n
        if scheme == "mrt":
            H = S.mrt_symbol(kx, ky, s_xx=s_xx, s_q=s_q)
            phi0, phi = fourier(f0, *m), fourier(got, *m)
        else:
            H = S.fd_symbol(kx, ky, s_xx=s_xx, s_e=1.0, stencil=int(scheme[2]))
            phi0 = np.array([fourier(a, *m) for a in init])
            phi = np.array([fourier(a, *m) for a in got])
        pred = np.linalg.matrix_power(H, steps) @ phi0
        err = np.max(np.abs(phi - pred)) / np.max(np.abs(pred))
        worst = max(worst, err)
    print(f"  256^2 FP32 RMS 1e-6 {scheme}: worst mode error after 10000 steps {worst:.2e}")
    assert worst < 2e-4


@pytest.mark.parametrize("scheme", ["fd3", "mrt"])
def test_poiseuille_channel_16384x1024(F, scheme):
    """FP32 channel 16384 x 1024 started from the analytic parabola: after 2000 steps the
    profile is x-invariant, equals the FP64 oracle's on an 8-column channel, and stays
    within 5e-6 of the parabola (relative L2; the FP64 oracle is within 5e-7)."""
    nx, ny, steps = 16384, 1024, 2000
    nu = 1 / math.sqrt(108)
    s_xx = O.rate_from_viscosity(nu)
    r, x, y, Fx = W.poiseuille_profile(nx, ny, nu, 0.05)
    exact = x[:, 0].copy()
    kw = dict(bc="walls", dtype="f32", s_xx=s_xx, force=(Fx, 0.0))
    if scheme == "mrt":
        sim = F.FdLbm(nx, ny, scheme="mrt", quartic=True, **kw)
    else:
        sim = F.FdLbm(nx, ny, scheme="fd", stencil=3, s_e=1.0, **kw)
    sim.set_state(r, x, y)
    sim.step(steps)
    gr, gx, gy = sim.get_state()
    sim.close()
    spread = float(np.max(np.abs(gx - gx[:, :1])))
    assert spread < 1e-7 * 0.05, spread
    u = gx.mean(axis=1) + Fx / 2
    r8, x8, y8 = (a[:, :8].copy() for a in (r, x, y))
    if scheme == "mrt":
        want = O.mrt_moments(O.mrt_run(O.mrt_init(r8, x8, y8), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx),
                                       walls=True, fx=Fx))[1][:, 0] + Fx / 2
    else:
        want = O.fd_run(r8, x8, y8, steps, s_xx=s_xx, s_e=1.0, stencil=3, walls=True, fx=Fx)[1][:, 0] + Fx / 2
    err_oracle = np.linalg.norm(u - want) / np.linalg.norm(want)
    err_parab = np.linalg.norm(u - exact) / np.linalg.norm(exact)
    print(f"  {scheme}: rel L2 vs oracle {err_oracle:.2e}, vs parabola {err_parab:.2e}")
    assert err_oracle < 1e-5
    assert err_parab < 5e-6


def test_decaying_flow_8192_2000_steps(F):
    """FP32 keeps the FP64 result to 1e-5 over 2000 steps (measured 3e-7: the update adds
    small differences to the stored state, so no rounding bias accumulates).  FP16 storage
    is limited by its 11-bit significand: on this slowly varying flow a step changes a value
    by about one FP16 unit, and after 2000 steps the relative L2 error is 2.9e-2 (5e-4 after
    12 steps, see test_gpu_sweep.py); the bound 5e-2 states that measurement."""
    n, steps = 8192, 2000
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    s_xx = O.rate_from_viscosity(0.02)
    ref = run_gpu(F, init, steps, scheme="fd", stencil=3, dtype="f64", s_xx=s_xx, s_e=1.0)
    e32 = rel_l2(run_gpu(F, init, steps, scheme="fd", stencil=3, dtype="f32", s_xx=s_xx, s_e=1.0), ref)
    e16 = rel_l2(run_gpu(F, init, steps, scheme="fd", stencil=3, dtype="f16", s_xx=s_xx, s_e=1.0), ref)
    e16sr = rel_l2(run_gpu(F, init, steps, scheme="fd", stencil=3, dtype="f16sr", s_xx=s_xx, s_e=1.0), ref)
    print(f"  8192^2 2000 steps: FP32 rel L2 {e32:.2e}, FP16 storage rel L2 {e16:.2e}, "
          f"FP16 stochastic rounding {e16sr:.2e} (vs FP64 GPU)")
    assert e32 < 1e-5
    assert e16 < 5e-2
    assert e16sr < 5e-2


def test_mrt_decaying_flow_8192_2000_steps(F):
    """MRT in FP32 keeps its FP64 result over the configuration's 2000 steps at 8192^2 (the
    collision adds the small change m* - m to the stored deviations)."""
    n, steps = 8192, 2000
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    s_xx = O.rate_from_viscosity(0.02)
    ref = run_gpu(F, init, steps, scheme="mrt", dtype="f64", s_xx=s_xx, quartic=True)
    got = run_gpu(F, init, steps, scheme="mrt", dtype="f32", s_xx=s_xx, quartic=True)
    err = math.sqrt(float(np.sum((got - ref) ** 2)) / float(np.sum(ref ** 2)))
    print(f"  8192^2 2000 steps: MRT FP32 populations rel L2 {err:.2e} (vs MRT FP64 GPU)")
    assert err < 1e-5


@pytest.mark.parametrize("scheme,dtype,tol", [("fd3", "f64", 1e-12), ("fd5", "f32", 1e-5), ("mrt", "f32", 1e-5),
                                              ("mrt", "f64", 1e-12)])
def test_full_size_band_other_schemes(F, scheme, dtype, tol):
    """8192 x 8192 decaying flow in the default launch configuration of each scheme: after 10
    steps, 128 rows against the oracle run on those rows plus their domain of dependence
    (3 rows per step for 5-point differences, 2 for 3-point, 1 for MRT)."""
    n, steps, rows, y0 = 8192, 10, 128, 5000
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    s_xx = O.rate_from_viscosity(0.02)
    if scheme == "mrt":
        m = steps + 1
        band = tuple(np.ascontiguousarray(a[y0 - m:y0 + rows + m]) for a in init)
        sim = F.FdLbm(n, n, scheme="mrt", dtype=dtype, s_xx=s_xx, quartic=True)
        sim.set_state(*init)
        sim.step(steps)
        got = sim.get_state()  # moments of the populations, reduced on the device
        sim.close()
        want = O.mrt_moments(O.mrt_run(O.mrt_init(*band), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx)))
    else:
        st = int(scheme[2])
        m = steps * (3 if st == 5 else 2)
        band = tuple(np.ascontiguousarray(a[y0 - m:y0 + rows + m]) for a in init)
        got = run_gpu(F, init, steps, scheme="fd", stencil=st, dtype=dtype, s_xx=s_xx, s_e=1.0)
        want = O.fd_run(*band, steps, s_xx=s_xx, s_e=1.0, stencil=st)
    err = rel_l2([g[y0:y0 + rows] for g in got], [w[m:m + rows] for w in want])
    print(f"  8192^2 {scheme} {dtype} band rel L2 {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_largest_grids_beyond_2_31_nodes(F, dtype):
    """65536 x 36864 = 2.4e9 nodes, so each plane holds more than 2^31 values (the ABI allows
    nx * ny up to 2^32).  A uniform state under a body force stays uniform, and the step
    adds exactly F to J at every node (section 1, Strang splitting; F a power of two, exact
    in FP16 too), so after k steps the FP64 diagnostics equal n k F exactly, which a node
    left out or visited twice anywhere in the grid would change.  The state starts at rest
    (fdlbm_create clears it), so no host array of that size is needed."""
    import torch

    nx, ny, steps = 65536, 36864, 6
    fx, fy = 2.0 ** -10, -(2.0 ** -11)
    n = nx * ny
    print(f"case largest grid {nx}x{ny} dtype={dtype}", flush=True)
    sim = F.FdLbm(nx, ny, dtype=dtype, stencil=3, s_xx=1.5, force=(fx, fy))
    sim.step(steps)
    d = sim.diagnostics()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    jx, jy = steps * fx, steps * fy
    print(f"  mass {d['mass']}, momentum ({d['mom_x']}, {d['mom_y']}), max |J| {d['max_abs_j']}")
    assert d["nonfinite"] == 0
    assert d["mass"] == 0.0
    assert d["mom_x"] == n * jx and d["mom_y"] == n * jy
    assert abs(d["max_abs_j"] - math.hypot(jx, jy)) <= 1e-15
    assert abs(d["kin_energy"] / (0.5 * n * (jx * jx + jy * jy)) - 1) < 1e-12


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("f64", 1e-13)])
def test_mrt_state_beyond_2_31_values(F, dtype, tol):
    """MRT on 16384 x 16384: the nine row-interleaved populations hold 2.4e9 values, so the
    element offsets of the upper rows pass 2^31 (past 2^34 bytes in FP64).  A uniform state at
    rest (fdlbm_create clears it) under a body force stays uniform, since propagation moves
    equal populations between equal nodes; after k steps every node must hold what one node
    of the FP64 oracle's 4 x 4 run holds (section 1, eqs. 1-2, Strang force).  Nodes in the
    first, middle and last rows are read straight from the state buffer at the documented
    element (9y + k) nx + x: equal to each other bit for bit, and to the oracle's node within
    `tol` of its largest population; the FP64 diagnostics equal n times the node's moments."""
    import torch

    nx = ny = 16384
    steps, fx, fy, s_xx = 6, 2.0 ** -10, -(2.0 ** -11), 1.5
    n = nx * ny
    print(f"case MRT {nx}x{ny} dtype={dtype} ({9 * n} values per state)", flush=True)
    sim = F.FdLbm(nx, ny, scheme="mrt", dtype=dtype, s_xx=s_xx, quartic=True, force=(fx, fy))
    sim.step(steps)
    d = sim.diagnostics()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    buf = (sim.buffers.state_a if steps % 2 == 0 else sim.buffers.state_b).view(tdt)
    nodes = [(0, 0), (nx - 1, ny // 2), (nx // 2, ny - 1), (nx - 1, ny - 1)]
    vals = np.array([[buf[(9 * y + k) * nx + x].item() for k in range(9)] for x, y in nodes])
    sim.close()
    del sim, buf
    torch.cuda.empty_cache()
    want = O.mrt_run(np.zeros((9, 4, 4)), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx), fx=fx, fy=fy)[:, 0, 0]
    scale = np.abs(want).max()
    print(f"  node populations {vals[0]}, oracle {want}")
    assert np.array_equal(vals, np.broadcast_to(vals[0], vals.shape))
    assert np.abs(vals[0] - want).max() <= tol * scale
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
    node = vals[0].astype(np.float64)
    assert d["nonfinite"] == 0
    for key, v in (("mass", node.sum()), ("mom_x", ex @ node), ("mom_y", ey @ node)):
        assert abs(d[key] - n * v) <= 1e-12 * n * scale, (key, d[key], n * v)


@pytest.mark.parametrize("stencil", [3, 5])
def test_relative_viscosity_curves_figs_2_3(F, stencil):
    """Section 3-a, Figs. 2 and 3: nu(k)/nu_0 at nu_0 = 0.01 for wave vectors along {1,0},
    {2,1} and {1,1}, from transverse waves on 64 x 64 grids (FP64, device projection A(t)
    between two times), against the shear root of the dispersion equation: equal to 1e-4
    relative for every point (the transverse start is not exactly the discrete eigenvector,
    so the other roots leave a trace of that size in A(t); the FP64 oracle run on the same
    points shows the same 4e-5), while the curves themselves move far from 1 at large k."""
    from oracle import symbol as S

    nu0, n = 0.01, 64
    s_xx = O.rate_from_viscosity(nu0)
    worst, spread = 0.0, 0.0
    for d in ((1, 0), (2, 1), (1, 1)):
        for m in (1, 2, 3, 4, 6):
            mx, my = m * d[0], m * d[1]
            kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
            k2 = kx * kx + ky * ky
            t1 = int(round(0.2 / (nu0 * k2)))
            t2 = t1 + int(round(1.0 / (nu0 * k2)))
            r, jx, jy = W.shear_wave(n, n, 1e-6, mx, my)
            sim = F.FdLbm(n, n, dtype="f64", stencil=stencil, s_xx=s_xx)
            sim.set_state(r, jx, jy)
            sim.set_mode(jx, jy)
            sim.step(t1)
            a1 = sim.mode_projection()
            sim.step(t2 - t1)
            a2 = sim.mode_projection()
            sim.close()
            rel = -math.log(a2 / a1) / (t2 - t1) / k2 / nu0
            want = S.nu_of_k(math.sqrt(k2), math.atan2(ky, kx), "fd", s_xx=s_xx, stencil=stencil) / nu0
            print(f"  FD{stencil} {d} k={math.sqrt(k2):.3f}: nu(k)/nu0 {rel:.6f} (dispersion {want:.6f})")
            worst = max(worst, abs(rel / want - 1))
            spread = max(spread, abs(want - 1))
    print(f"  FD{stencil}: worst relative difference {worst:.1e}, curves reach {spread:.3f} from 1")
    assert worst < 1e-4
    assert spread > (1.0 if stencil == 3 else 0.3)


@pytest.mark.parametrize("dtype,bound", [("f64", 1e-15), ("f32", 1e-8), ("f16", 1e-3), ("f16sr", 1e-4)])
def test_conservation_8192_2000_steps(F, dtype, bound):
    """Section 1 (eq. 2): total mass and momentum are invariants of the periodic step.  On the
    8192 x 8192 decaying flow over 2000 steps, the FP64 sums of the stored state move by less
    than `bound` relative to sum |field|: what remains is the random walk of the per-node
    rounding, with no systematic drift (summing the nine arriving populations instead would
    drift by about 3e-8 of the field per step in FP32): measured 8e-19 (FP64) and 2e-10
    (FP32).  FP16 storage is not conservative: an increment below half a unit of the stored
    deviation is lost, and on a slowly varying field the losses are correlated from step to
    step, so its stated bound is the measured 3e-4 of the mass with a margin."""
    n, steps = 8192, 2000
    init = W.decaying_flow(n=n, seed=4, kmax=32, amp=0.02)
    scale = [float(np.sum(np.abs(a))) for a in init]
    sim = F.FdLbm(n, n, dtype=dtype, stencil=3, s_xx=O.rate_from_viscosity(0.02))
    sim.set_state(*init)
    d0 = sim.diagnostics()
    sim.step(steps)
    d1 = sim.diagnostics()
    sim.close()
    drift = [abs(d1[q] - d0[q]) / s for q, s in zip(("mass", "mom_x", "mom_y"), scale)]
    print(f"  {dtype}: relative drift of mass, momentum after {steps} steps: "
          + ", ".join(f"{x:.2e}" for x in drift))
    assert d1["nonfinite"] == 0
    assert max(drift) < bound


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
@pytest.mark.parametrize("dtype,amp,tol", [("f64", 1e-6, 1.5e-3), ("f32", 1e-4, 3e-3)])
@pytest.mark.parametrize("direction", [(1, 0), (1, 1)])
def test_galilean_damping_in_a_mean_flow(F, scheme, dtype, amp, tol, direction):
    """Sections 1-a and 2: a transverse wave carried by a uniform flow V parallel to its wave
    vector is damped with nu (1 - 3 V^2) by D2Q9 MRT and by FD-LBM alike (the theta terms
    give FD-LBM the lattice Boltzmann behaviour, where LW-ACM has nu - V^2/2).  Along an axis
    the factor comes from the velocity-cubic terms of theta_XY, along a diagonal from those of
    theta_XX.  The rate is read from the wave's Fourier amplitude in the device state at two
    times."""
    nu = 0.05
    s_xx = O.rate_from_viscosity(nu)
    nx, ny, t1, t2 = (128, 8, 200, 1200) if direction == (1, 0) else (48, 48, 100, 500)
    k = 2 * math.pi * math.hypot(direction[0] / nx, direction[1] / ny)
    t = np.array([-direction[1], direction[0]]) / math.hypot(*direction)
    kw = dict(scheme="mrt", quartic=True) if scheme == "mrt" else dict(scheme="fd", stencil=int(scheme[2]))
    rates = {}
    for V in (0.0, 0.1, 0.2):
        init = W.shear_wave(nx, ny, amp, direction[0], direction[1], V=V)
        sim = F.FdLbm(nx, ny, dtype=dtype, s_xx=s_xx, s_e=1.0, **kw)
        sim.set_state(*init)
        sim.step(t1)
        m1 = sim.get_state()
        sim.step(t2 - t1)
        m2 = sim.get_state()
        sim.close()
        a1 = abs(fourier(t[0] * m1[1] + t[1] * m1[2], *direction))
        a2 = abs(fourier(t[0] * m2[1] + t[1] * m2[2], *direction))
        rates[V] = math.log(a1 / a2) / (t2 - t1) / k ** 2
    for V in (0.1, 0.2):
        print(f"  {scheme} {dtype} {direction} V={V}: nu_eff/nu {rates[V] / rates[0.0]:.5f} "
              f"(1 - 3 V^2 = {1 - 3 * V * V:.5f})")
        assert abs(rates[V] / rates[0.0] - (1 - 3 * V * V)) < tol


@pytest.mark.parametrize("stencil", [3, 5])
def test_table1_hyperviscosity_from_simulation(F, stencil):
    """Section 3-a, Table 1: the hyperviscosity nu_2 at s_xx = 1.85, measured as the paper did,
    from simulations: transverse waves along {1,0}, {2,1} and {1,1} at five small wave numbers
    each (FP64, device projection between two times), nu(k) - nu_0 fitted by
    nu_2 k^2 + nu_4 k^4.  The fits match the printed entries to 1 % (three points) and 5 %
    (five points, whose nu_2 is 36 times smaller); measured, they agree to the printed
    digits except at {2,1}, which lies at 26.565 degrees, the printed row at 26.6."""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_hyperviscosity.json")))
    s_xx = g["s_xx"]
    nu0 = (1.0 / s_xx - 0.5) / 3.0
    cases = (((1, 0), 128), ((2, 1), 256), ((1, 1), 181))
    for (d, n), printed in zip(cases, g["nu2"][str(stencil)]):
        ks, ys = [], []
        for m in (2, 3, 4, 5, 6):
            mx, my = m * d[0], m * d[1]
            kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
            k2 = kx * kx + ky * ky
            t1 = int(round(0.2 / (nu0 * k2)))
            t2 = t1 + int(round(1.0 / (nu0 * k2)))
            r, jx, jy = W.shear_wave(n, n, 1e-6, mx, my)
            sim = F.FdLbm(n, n, dtype="f64", stencil=stencil, s_xx=s_xx)
            sim.set_state(r, jx, jy)
            sim.set_mode(jx, jy)
            sim.step(t1)
            a1 = sim.mode_projection()
            sim.step(t2 - t1)
            a2 = sim.mode_projection()
            sim.close()
            ks.append(math.sqrt(k2))
            ys.append(-math.log(a2 / a1) / (t2 - t1) / k2 - nu0)
        ks = np.array(ks)
        nu2 = np.linalg.lstsq(np.stack([ks ** 2, ks ** 4], 1), np.array(ys), rcond=None)[0][0]
        print(f"  FD{stencil} {d}: nu_2 from simulation {nu2:.5f}, Table 1 {printed:.5f}")
        tol = 0.01 * abs(printed) + 3e-5 if stencil == 3 else 0.05 * abs(printed)
        assert abs(nu2 - printed) < tol


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
@pytest.mark.parametrize("s_e", [1.0, 1.5])
def test_sound_speed_and_damping(F, scheme, s_e):
    """Sections 1-a and 2: a sound wave travels at c_s = 1/sqrt(3) and is damped at
    Gamma_s = (nu + zeta) k^2 / 2, zeta = (1/s_e - 1/2)/3 the bulk viscosity, in MRT and in
    FD-LBM alike.  A right-moving wave (drho = a cos kx, Jx = c_s drho) on a 128^2 grid, FP64,
    is followed through the phase and modulus of the Fourier coefficient of the device state;
    both equal the acoustic root of the amplification matrix (to 1e-5 and 1e-3) and the closed
    forms (to 5e-4 and 1.5 %), so the step uses s_e where the theory puts it."""
    from oracle import symbol as S

    n, m, amp, s_xx = 128, 2, 1e-6, 1.8
    k = 2 * math.pi * m / n
    nu, zeta, cs = (1 / s_xx - 0.5) / 3, (1 / s_e - 0.5) / 3, 1 / math.sqrt(3)
    x = np.arange(n)
    r = np.tile(amp * np.cos(k * x), (n, 1))
    init = (r, cs * r, np.zeros((n, n)))
    kw = dict(scheme="mrt", quartic=True) if scheme == "mrt" else dict(scheme="fd", stencil=int(scheme[2]))
    sim = F.FdLbm(n, n, dtype="f64", s_xx=s_xx, s_e=s_e, **kw)
    sim.set_state(*init)
    e = np.exp(-1j * k * x)
    ts, cs_t = [], []
    for t in range(0, 1001, 10):
        if t >= 100:
            ts.append(t)
            cs_t.append(np.sum(sim.get_state()[0] * e[None, :]))
        sim.step(10)
    sim.close()
    ts, c = np.array(ts), np.array(cs_t)
    omega = -np.polyfit(ts, np.unwrap(np.angle(c)), 1)[0]
    gamma = -np.polyfit(ts, np.log(np.abs(c)), 1)[0]
    sym_kw = dict(s_xx=s_xx, s_e=s_e)
    if scheme == "mrt":
        sym_kw["s_q"] = O.quartic_s_q(s_xx)
    else:
        sym_kw["stencil"] = int(scheme[2])
    root = [z for z in S.sound_gammas(k, 0.0, "mrt" if scheme == "mrt" else "fd", **sym_kw) if z.imag > 0][0]
    print(f"  {scheme} s_e={s_e}: c {omega / k:.6f} (root {root.imag / k:.6f}, 1/sqrt3 {cs:.6f}); "
          f"Gamma/k^2 {gamma / k / k:.5f} (root {root.real / k / k:.5f}, (nu+zeta)/2 {(nu + zeta) / 2:.5f})")
    assert abs(omega / k - root.imag / k) < 1e-5
    assert abs(gamma / root.real - 1) < 1e-3
    assert abs(omega / k / cs - 1) < 5e-4
    assert abs(gamma / k / k / ((nu + zeta) / 2) - 1) < 0.015


def _device_flow_symbol(F, n, mode, V, s_e, stencil, s_xx=1.6, eps=1e-6):
    """3x3 amplification matrix of one FP64 device step about the uniform flow rho = 1, J = V,
    by central differences: column j is the response at the wave's mode to a plane wave of
    amplitude eps in field j."""
    nx, ny = n
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    phase = 2 * np.pi * (mode[0] * x / nx + mode[1] * y / ny)
    H = np.zeros((3, 3), dtype=complex)
    sim = F.FdLbm(nx, ny, scheme="fd", stencil=stencil, dtype="f64", s_xx=s_xx, s_e=s_e)
    for j in range(3):
        resp = []
        for sgn in (1.0, -1.0):
            f = [np.zeros((ny, nx)), np.full((ny, nx), V[0]), np.full((ny, nx), V[1])]
            f[j] = f[j] + sgn * eps * np.cos(phase)
            sim.set_state(*f)
            sim.step(1)
            resp.append(sim.get_state())
        for i in range(3):
            H[i, j] = np.sum((resp[0][i] - resp[1][i]) / (2 * eps) * np.exp(-1j * phase)) * 2 / (nx * ny)
    sim.close()
    return H


def _mean_acoustic_damping(H, kx, ky):
    z, vec = np.linalg.eig(H)
    k = math.hypot(kx, ky)
    g = [-np.log(z[i]).real for i in range(3)
         if (abs(vec[0, i]) + abs(vec[1, i] * kx / k + vec[2, i] * ky / k)) / np.linalg.norm(vec[:, i]) > 0.5]
    assert len(g) == 2, g
    return 0.5 * (g[0] + g[1])


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("vdir", [(1, 0), (1, 1)])
def test_bulk_viscosity_in_a_mean_flow(F, stencil, vdir):
    """Section 2: in a mean flow V the bulk viscosity is zeta (1 - 3V^2).  The device step's
    own amplification matrix about J = V (FP64, central differences of one step) equals the
    oracle's symbol at s_e = 1.4, where the velocity-cubic term of theta_E acts; and the zeta
    coefficient of its sound damping, extrapolated to k = 0 from wavelengths 64 and 128
    (zeta = 0.1 and 0.2), is (1 - 3V^2)/2."""
    V = 0.15
    u = np.array(vdir, dtype=float) / math.hypot(*vdir)
    vel = (V * u[0], V * u[1])
    H = _device_flow_symbol(F, (32, 32), (1, 1), vel, 1.4, stencil)
    want = S.fd_symbol(2 * math.pi / 32, 2 * math.pi / 32, s_xx=1.6, s_e=1.4, stencil=stencil, vx=vel[0], vy=vel[1])
    dev = float(np.max(np.abs(H - want)))
    b = []
    for n in (64, 128):
        k = 2 * math.pi / n
        g = [_mean_acoustic_damping(_device_flow_symbol(F, (n, 8), (1, 0), vel, 1 / (0.5 + 3 * z), stencil), k, 0.0)
             / (k * k) for z in (0.1, 0.2)]
        b.append((g[1] - g[0]) / 0.1)
    two_b = 2 * (4 * b[1] - b[0]) / 3
    print(f"  FD{stencil} V={vel}: |H - symbol| {dev:.1e}; 2B {two_b:.6f} (1 - 3V^2 = {1 - 3 * V * V:.6f})")
    assert dev < 1e-8
    assert abs(two_b - (1 - 3 * V * V)) < 5e-5


def test_d2q9_relative_viscosity_fig5(F):
    """Section 3-a, Fig. 5: nu(k)/nu_0 of the D2Q9 lattice Boltzmann model along {1,0}, {2,1},
    {1,1}, whose largest error the caption puts at 8 %.  The curve is not printed, nor are the
    model's rates and the k range; reading: nu_0 = 0.01 as in Figs. 2-4, k up to 1, and BGK
    (all rates equal), whose largest error over that range is 8.6 % (along {1,0} at k = 1).
    Measured on the device with the MRT kernel (FP64, 64^2 grids, two-time projection past the
    initial layer), every point equals the shear root of the amplification matrix to 1e-4; the
    largest error is 7-10 % for BGK and below 3 % for the quartic MRT."""
    from oracle import symbol as S

    nu0, n = 0.01, 64
    s = O.rate_from_viscosity(nu0)
    models = {"bgk": dict(s_xx=s, s_e=s, s_q=s, s_eps=s), "quartic": dict(s_xx=s, s_q=O.quartic_s_q(s))}
    points = [((1, 0), m) for m in (2, 4, 6, 8, 10)] + [((2, 1), m) for m in (1, 2, 3, 4)] + \
             [((1, 1), m) for m in (2, 4, 6, 7)]
    worst = {}
    for name, rates in models.items():
        worst[name] = 0.0
        for d, m in points:
            mx, my = m * d[0], m * d[1]
            kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
            k2 = kx * kx + ky * ky
            t1 = max(100, int(round(0.2 / (nu0 * k2))))
            t2 = t1 + int(round(1.0 / (nu0 * k2)))
            r, jx, jy = W.shear_wave(n, n, 1e-6, mx, my)
            sim = F.FdLbm(n, n, scheme="mrt", dtype="f64", **rates)
            sim.set_state(r, jx, jy)
            sim.set_mode(jx, jy)
            sim.step(t1)
            a1 = sim.mode_projection()
            sim.step(t2 - t1)
            a2 = sim.mode_projection()
            sim.close()
            rel = -math.log(a2 / a1) / (t2 - t1) / k2 / nu0
            want = S.nu_of_k(math.sqrt(k2), math.atan2(ky, kx), "mrt", **rates) / nu0
            assert abs(rel / want - 1) < 1e-4, (name, d, m, rel, want)
            worst[name] = max(worst[name], abs(rel - 1))
        print(f"  D2Q9 {name}: largest |nu(k)/nu0 - 1| for k <= 1: {worst[name]:.4f}")
    assert 0.07 < worst["bgk"] < 0.10
    assert worst["quartic"] < 0.03
