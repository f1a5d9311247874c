"""The layout of the caller-owned state buffers that the C ABI documents (include/fdlbm.h,
include/fdlbm3d.h), checked from the caller's side:

* two-dimensional steps: F fields, node (x, y) of field f at element (F*y + f)*nx + x, with
  F = 3 (drho, Jx, Jy) for FD-LBM and LW-ACM and F = 9 (the populations f_k - w_k in velocity
  order) for MRT;
* D3Q19: four planes (drho, Jx, Jy, Jz), node (x, y, z) at (z*ny + y)*nx + x.

A state uploaded through the ABI must sit in the buffer exactly there, a buffer written by
hand in that layout must read back through the ABI unchanged, and the allocation-free
diagnostics must read such a buffer as the scheme's state."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NP = {"f64": np.float64, "f32": np.float32, "f16": np.float16, "f16sr": np.float16}
# D2Q9 velocities in the order of section 1 (e_0 .. e_8)
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


def _fields(nf, ny, nx, seed):
    """nf host planes with values exactly representable in FP32 (so that FP16 storage rounds
    them once, on the device as in NumPy)."""
    rng = np.random.default_rng(seed)
    return (0.02 * (2 * rng.random((nf, ny, nx)) - 1)).astype(np.float32).astype(np.float64)


def _interleaved(planes):
    """(F, ny, nx) planes -> the documented row-interleaved element order."""
    return np.ascontiguousarray(np.transpose(planes, (1, 0, 2))).reshape(-1)


def _buffer(sim, dtype, count):
    import torch

    tdt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "f16sr": torch.float16}[dtype]
    return sim.buffers.state_a.view(tdt)[:count]


CASES_2D = [("fd", "f64"), ("fd", "f32"), ("fd", "f16"), ("fd", "f16sr"), ("lwacm", "f32"), ("mrt", "f64"),
            ("mrt", "f32")]


@pytest.mark.parametrize("scheme,dtype", CASES_2D)
def test_uploaded_state_is_row_interleaved(F, scheme, dtype):
    nx, ny = 37, 21   # odd width, ragged against every lane group
    print(f"  layout upload {scheme} {dtype} {nx}x{ny}", flush=True)
    sim = F.FdLbm(nx, ny, scheme=scheme, dtype=dtype, s_xx=1.2, s_e=1.0)
    nf = 9 if scheme == "mrt" else 3
    planes = _fields(nf, ny, nx, seed=nf * 100 + len(dtype))
    if scheme == "mrt":
        sim.set_populations(planes)
    else:
        sim.set_state(*planes)
    got = _buffer(sim, dtype, nf * nx * ny).cpu().numpy()
    want = _interleaved(planes).astype(NP[dtype])
    assert np.array_equal(got, want)
    sim.close()


@pytest.mark.parametrize("scheme,dtype", CASES_2D)
def test_hand_written_buffer_reads_back(F, scheme, dtype):
    import torch

    nx, ny = 37, 21
    print(f"  layout read-back {scheme} {dtype} {nx}x{ny}", flush=True)
    sim = F.FdLbm(nx, ny, scheme=scheme, dtype=dtype, s_xx=1.2, s_e=1.0)
    nf = 9 if scheme == "mrt" else 3
    planes = _fields(nf, ny, nx, seed=nf * 10 + len(dtype))
    stored = _interleaved(planes).astype(NP[dtype])
    buf = _buffer(sim, dtype, stored.size)
    buf.copy_(torch.from_numpy(stored).to(buf.device))
    torch.cuda.synchronize()
    back = sim.get_populations() if scheme == "mrt" else np.stack(sim.get_state())
    assert np.array_equal(back, planes.astype(NP[dtype]).astype(np.float64))
    sim.close()


@pytest.mark.parametrize("scheme,dtype", CASES_2D)
def test_static_diagnostics_read_the_documented_layout(F, scheme, dtype):
    """fdlbm_diagnostics_static on a buffer the caller filled in the documented layout, against
    the same sums in NumPy (FP64 sums in another order: agreement to rounding)."""
    import torch

    nx, ny = 37, 21
    print(f"  layout static diagnostics {scheme} {dtype} {nx}x{ny}", flush=True)
    nf = 9 if scheme == "mrt" else 3
    planes = _fields(nf, ny, nx, seed=nf + len(dtype)).astype(NP[dtype]).astype(np.float64)
    params = F.make_params(nx, ny, scheme=scheme, dtype=dtype, s_xx=1.2, s_e=1.0)
    state = torch.from_numpy(_interleaved(planes).astype(NP[dtype])).cuda()
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    F.fdlbm_diagnostics_static(params, state.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if scheme == "mrt":
        dr = planes.sum(axis=0)
        jx = np.tensordot(EX, planes, axes=1)
        jy = np.tensordot(EY, planes, axes=1)
    else:
        dr, jx, jy = planes
    j2 = jx * jx + jy * jy
    want = [dr.sum(), jx.sum(), jy.sum(), 0.5 * (j2 / (1.0 + dr)).sum(), np.sqrt(j2).max()]
    scale = [np.abs(dr).sum(), np.abs(jx).sum(), np.abs(jy).sum(), want[3], want[4]]
    for k, (g, w, s) in enumerate(zip(got[:5], want, scale)):
        assert abs(g - w) <= 1e-12 * s, (k, g, w)
    assert got[5] == 0 and got[6] == 0 and got[7] == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_d3q19_state_is_four_planes(F, dtype):
    import torch

    nx, ny, nz = 19, 7, 5
    print(f"  layout D3Q19 {dtype} {nx}x{ny}x{nz}", flush=True)
    sim = F.FdLbm3D(nx, ny, nz, dtype=dtype, s_nu=1.2, s_e=1.0)
    rng = np.random.default_rng(3)
    planes = (0.02 * (2 * rng.random((4, nz, ny, nx)) - 1)).astype(np.float32).astype(np.float64)
    sim.set_state(*planes)
    count = 4 * nx * ny * nz
    tdt = torch.float64 if dtype == "f64" else torch.float32
    got = sim.buffers.state_a.view(tdt)[:count].cpu().numpy()
    assert np.array_equal(got, planes.reshape(-1).astype(NP[dtype]))
    sim.close()
