"""Batched FD-LBM path: every instance evolves exactly as the same grid alone (bit for bit),
the one-launch-per-step, per-instance and graph-replayed paths agree bit for bit, and the
device FP64 correlation samples A(t) match the host computation and the oracle."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

SPECS = [(33, 40, 1.6, 1.0), (64, 64, 1.2, 1.1), (100, 37, 1.85, 1.0), (8, 8, 1.5, 1.0), (250, 130, 1.9, 1.0),
         (61, 9, 1.3, 1.2)]


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


def initial(i, nx, ny):
    return W.random_state(nx, ny, seed=100 + i, amp=0.02)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
def test_batch_instances_equal_single_grids_bitwise(F, dtype):
    steps = 20
    batch = F.FdLbmBatch(SPECS, dtype=dtype, max_samples=4)
    for i, (nx, ny, _, _) in enumerate(SPECS):
        batch.set_state(i, *initial(i, nx, ny))
    batch.step(steps, sample_every=10, use_graph=True)
    for i, (nx, ny, s_xx, s_e) in enumerate(SPECS):
        print(f"case batch dtype={dtype} instance={i} shape=({nx},{ny})", flush=True)
        sim = F.FdLbm(nx, ny, dtype=dtype, stencil=3, s_xx=s_xx, s_e=s_e, kernel="sweep", lane_cols=1, tile_rows=8)
        sim.set_state(*initial(i, nx, ny))
        sim.step(steps)
        want = sim.get_state()
        sim.close()
        got = batch.get_state(i)
        for u, v in zip(got, want):
            assert np.array_equal(u, v)
    batch.close()


def test_batch_paths_agree_bitwise(F):
    runs = {}
    for mode in ("graph", "direct", "per_instance"):
        b = F.FdLbmBatch(SPECS, dtype="f32", max_samples=8)
        for i, (nx, ny, _, _) in enumerate(SPECS):
            b.set_state(i, *initial(i, nx, ny))
        if mode == "per_instance":
            b.step_per_instance(30)
            amps = None
        else:
            b.step(30, sample_every=5, use_graph=mode == "graph")
            amps = b.amplitudes()
        runs[mode] = ([b.get_state(i) for i in range(len(SPECS))], amps)
        b.close()
    for mode in ("direct", "per_instance"):
        for sa, sb in zip(runs["graph"][0], runs[mode][0]):
            for u, v in zip(sa, sb):
                assert np.array_equal(u, v), mode
    assert runs["graph"][1].shape == (len(SPECS), 6)
    assert np.array_equal(runs["graph"][1], runs["direct"][1])


def test_batch_amplitudes_match_host_and_oracle(F):
    steps, every = 40, 8
    b = F.FdLbmBatch(SPECS, dtype="f64", max_samples=10)
    for i, (nx, ny, _, _) in enumerate(SPECS):
        b.set_state(i, *initial(i, nx, ny))
    b.step(steps, sample_every=every, use_graph=True)
    amps = b.amplitudes()
    assert amps.shape == (len(SPECS), steps // every)
    for i, (nx, ny, s_xx, s_e) in enumerate(SPECS):
        r0, x0, y0 = initial(i, nx, ny)
        _, x, y = b.get_state(i)
        host = np.sum(x * x0 + y * y0) / np.sum(x0 * x0 + y0 * y0)
        assert abs(amps[i, -1] - host) < 1e-12 * max(1.0, abs(host))
        st = (r0, x0, y0)
        for s in range(steps // every):
            st = O.fd_run(*st, every, s_xx=s_xx, s_e=s_e, stencil=3)
            want = np.sum(st[1] * x0 + st[2] * y0) / np.sum(x0 * x0 + y0 * y0)
            assert abs(amps[i, s] - want) < 1e-12, (i, s)
    b.close()


def test_batch_fitted_viscosity_matches_symbol(F):
    """Shear waves jx = 0.01 sin(2 pi m y / N) of several sizes and viscosities: the decay
    rate fitted to the device A(t) samples equals the amplification matrix's shear root."""
    from oracle import symbol as S

    specs, modes = [], []
    for n, nu, m in ((48, 0.05, 1), (96, 0.02, 2), (128, 0.1, 1), (40, 0.005, 1)):
        specs.append((n, n, O.rate_from_viscosity(nu), 1.0))
        modes.append(m)
    steps, every = 1000, 10
    b = F.FdLbmBatch(specs, dtype="f32", max_samples=steps // every)
    for i, ((n, _, _, _), m) in enumerate(zip(specs, modes)):
        b.set_state(i, *W.shear_wave_y(n, n, 0.01, m))
    b.step(steps, sample_every=every, use_graph=True)
    amps = b.amplitudes()
    b.close()
    t = np.arange(1, steps // every + 1) * every
    for i, ((n, _, s_xx, _), m) in enumerate(zip(specs, modes)):
        g = -np.polyfit(t[10:], np.log(amps[i, 10:]), 1)[0]
        g_sym = S.shear_gamma(0.0, 2 * math.pi * m / n, s_xx=s_xx, stencil=3).real
        print(f"  instance {i}: fitted Gamma {g:.6e}, symbol {g_sym:.6e}")
        assert abs(g / g_sym - 1) < 2e-4
