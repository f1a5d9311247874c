"""The allocation-free diagnostics entry point (static device scratch) against the one that
takes the context's scratch buffer: identical FP64 results, on two calls in a row, the second
on a smaller grid, for FD-LBM, MRT and FP16 storage, with and without a reference mode."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SLOTS = ("mass", "mom_x", "mom_y", "kin_energy", "max_abs_j", "proj_num", "proj_den", "nonfinite")


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


def _static(F, sim, j0=None):
    """fdlbm_diagnostics_static on the buffer holding the context's current state."""
    import torch

    state = sim.buffers.state_a if sim.steps_since_create % 2 == 0 else sim.buffers.state_b
    out = torch.full((8,), float("nan"), dtype=torch.float64, device=state.device)
    if j0 is not None:
        jx = torch.from_numpy(np.ascontiguousarray(j0[0])).to(state.device)
        jy = torch.from_numpy(np.ascontiguousarray(j0[1])).to(state.device)
        F.fdlbm_diagnostics_static(sim.params, state.data_ptr(), out.data_ptr(), jx.data_ptr(), jy.data_ptr(),
                                   sim.stream.cuda_stream)
    else:
        F.fdlbm_diagnostics_static(sim.params, state.data_ptr(), out.data_ptr(), stream=sim.stream.cuda_stream)
    sim.stream.synchronize()
    return out.cpu().numpy()


class Sim:
    """An FdLbm that counts every step since creation (the buffer of the current state)."""

    def __init__(self, F, nx, ny, **kw):
        self.sim = F.FdLbm(nx, ny, **kw)
        self.steps_since_create = 0
        self.buffers, self.params, self.stream = self.sim.buffers, self.sim.params, self.sim.stream

    def step(self, n):
        self.sim.step(n)
        self.steps_since_create += n


@pytest.mark.parametrize("kw", [dict(scheme="fd", dtype="f32"), dict(scheme="fd", dtype="f64"),
                                dict(scheme="fd", dtype="f16"), dict(scheme="mrt", dtype="f32", quartic=True)])
def test_static_diagnostics_equal_the_scratch_ones(F, kw):
    shapes = [(300, 200, 3), (70, 45, 2)]   # second call: a smaller grid
    for nx, ny, steps in shapes:
        print(f"  static diagnostics {kw} {nx}x{ny}", flush=True)
        r, x, y = W.random_state(nx, ny, seed=nx + ny, amp=0.02)
        s = Sim(F, nx, ny, s_xx=1.3, s_e=1.1, **kw)
        s.sim.set_state(r, x, y)
        s.step(steps)
        want = s.sim.diagnostics()
        got = _static(F, s)
        for q, name in enumerate(SLOTS):
            assert got[q] == float(want[name]), (name, got[q], want[name])
        # with a reference mode J0 (the correlation A(t) of section 3-a)
        j0 = (np.sin(np.arange(nx) * 0.1)[None, :] * np.ones((ny, 1)), np.cos(np.arange(ny) * 0.2)[:, None] * np.ones((1, nx)))
        s.sim.set_mode(*j0)
        want = s.sim.diagnostics()
        got = _static(F, s, j0)
        for q, name in enumerate(SLOTS):
            assert got[q] == float(want[name]), (name, got[q], want[name])
        assert got[6] > 0
        s.sim.close()


def test_static_diagnostics_reject_bad_arguments(F):
    import torch

    p = F.make_params(64, 48, dtype="f32", s_xx=1.5)
    buf = torch.zeros(3 * 64 * 48, dtype=torch.float32, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FdlbmError) as e:
        F.fdlbm_diagnostics_static(F.make_params(64, 48, stencil=9), buf.data_ptr(), out.data_ptr())
    assert e.value.code == F.FDLBM_EINVAL
    with pytest.raises(F.FdlbmError):
        F.fdlbm_diagnostics_static(p, 0, out.data_ptr())
    with pytest.raises(F.FdlbmError):
        F.fdlbm_diagnostics_static(p, buf.data_ptr(), out.data_ptr(), j0x=buf.data_ptr())
    F.fdlbm_diagnostics_static(p, buf.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    assert out.cpu().numpy().tolist() == [0.0] * 8
