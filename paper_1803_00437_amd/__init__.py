"""MI355X (gfx950) FD-LBM, LW-ACM and MRT D2Q9 steps, and the FD-LBM step on D3Q19 -- thin
Python binding of libfdlbm.so.

The binding only marshals arguments: every step of the computation runs in the HIP
kernels of ``csrc/``, behind the C ABI declared in ``include/fdlbm.h`` and
``include/fdlbm3d.h``.  PyTorch is used
to allocate the caller-owned device buffers and to supply the HIP stream.

Module-level functions carry the C names (``fdlbm_create``, ``fdlbm_step``, ``mrt_step``, ``lwacm_step``,
``fdlbm_diagnostics``, ``fdlbm3d_step`` ...); :class:`FdLbm` and :class:`FdLbm3D` own the
buffers of one simulation.

There is no fallback: if ``_build/libfdlbm.so`` is missing, importing the binding's entry
points raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libfdlbm.so")

FDLBM_OK, FDLBM_EINVAL, FDLBM_ENOMEM, FDLBM_EDEVICE, FDLBM_EUNSTABLE = 0, -1, -2, -3, -4
SCHEME = {"fd": 0, "mrt": 1, "lwacm": 2}
BC = {"periodic": 0, "walls": 1, "disk": 2}
DTYPE = {"f64": 0, "f32": 1, "f16": 2, "f16sr": 3}
KERNEL = {"auto": 0, "reference": 1, "sweep": 2}

EXPORTED = (
    "fdlbm_workspace_bytes", "fdlbm_create", "fdlbm_set_state", "fdlbm_get_state",
    "fdlbm_set_populations", "fdlbm_get_populations", "fdlbm_step", "mrt_step", "lwacm_step",
    "fdlbm_diagnostics", "fdlbm_diagnostics_static", "fdlbm_set_mode", "fdlbm_mode_projection", "fdlbm_step_count",
    "fdlbm_set_step_count",
    "fdlbm_destroy", "fdlbm_strerror", "fdlbm_last_error", "fdlbm_rate_from_viscosity",
    "fdlbm_quartic_s_q", "fdlbm_device_copy", "fdlbm_autotune",
    "fdlbm_batch_workspace_bytes", "fdlbm_batch_create", "fdlbm_batch_set_state", "fdlbm_batch_get_state",
    "fdlbm_batch_step", "fdlbm_batch_step_per_instance", "fdlbm_batch_amplitudes", "fdlbm_batch_step_count",
    "fdlbm_batch_destroy", "fdlbm_batch_last_error", "fdlbm_batch_autotune",
    "fdlbm3d_workspace_bytes", "fdlbm3d_create", "fdlbm3d_set_state", "fdlbm3d_get_state", "fdlbm3d_step",
    "fdlbm3d_diagnostics", "fdlbm3d_step_count", "fdlbm3d_destroy", "fdlbm3d_last_error", "fdlbm3d_autotune",
)


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("stencil", ctypes.c_int32), ("bc", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("s_xx", ctypes.c_double), ("s_e", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_eps", ctypes.c_double), ("quartic", ctypes.c_int32),
        ("force_x", ctypes.c_double), ("force_y", ctypes.c_double),
        ("kernel", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("lane_cols", ctypes.c_int32), ("wall_xi", ctypes.c_double),
        ("disk_cx", ctypes.c_double), ("disk_cy", ctypes.c_double), ("disk_r", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("kin_energy", ctypes.c_double), ("max_abs_j", ctypes.c_double),
        ("proj_num", ctypes.c_double), ("proj_den", ctypes.c_double), ("nonfinite", ctypes.c_int64),
    ]


class Params3D(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("s_nu", ctypes.c_double), ("s_e", ctypes.c_double), ("kernel", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32), ("tile_planes", ctypes.c_int32),
    ]


class Diag3D(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("mom_z", ctypes.c_double), ("kin_energy", ctypes.c_double), ("max_abs_j", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
    ]


class Instance(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("s_xx", ctypes.c_double), ("s_e", ctypes.c_double)]


class FdlbmError(RuntimeError):
    def __init__(self, code, what):
        lib = _lib_or_none()
        msg = lib.fdlbm_strerror(code).decode() if lib else str(code)
        if code == FDLBM_EDEVICE and lib:
            last = lib.fdlbm3d_last_error if what.startswith("fdlbm3d") else lib.fdlbm_last_error
            msg += ": " + last().decode()
        super().__init__(f"{what}: {msg}")
        self.code = code


_LIB = None


def _lib_or_none():
    return _LIB


def load_library(path=LIB_PATH):
    """Load libfdlbm.so and declare its signatures.  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1803_00437_amd.build` "
                           "(there is no CPU fallback)")
    # torch ships its own HIP runtime and asks for it under a name that does not match the
    # soname of the system one.  Loaded first, torch's copy satisfies this library's
    # dependency, and both use one runtime; loaded after this library, torch would bring a
    # second runtime into the process and device buffers would not be shared.
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    vp, dp, i32, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int64
    P = ctypes.POINTER(Params)
    sig = {
        "fdlbm_workspace_bytes": (i32, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "fdlbm_create": (i32, [P, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "fdlbm_set_state": (i32, [vp, dp, dp, dp]),
        "fdlbm_get_state": (i32, [vp, dp, dp, dp]),
        "fdlbm_set_populations": (i32, [vp, dp]),
        "fdlbm_get_populations": (i32, [vp, dp]),
        "fdlbm_step": (i32, [vp, i64]),
        "mrt_step": (i32, [vp, i64]),
        "lwacm_step": (i32, [vp, i64]),
        "fdlbm_diagnostics": (i32, [vp, ctypes.POINTER(Diag)]),
        "fdlbm_diagnostics_static": (i32, [P, vp, vp, vp, vp, vp]),
        "fdlbm_set_mode": (i32, [vp, dp, dp]),
        "fdlbm_mode_projection": (i32, [vp, dp]),
        "fdlbm_step_count": (i64, [vp]),
        "fdlbm_set_step_count": (i32, [vp, i64]),
        "fdlbm_destroy": (None, [vp]),
        "fdlbm_strerror": (ctypes.c_char_p, [i32]),
        "fdlbm_last_error": (ctypes.c_char_p, []),
        "fdlbm_rate_from_viscosity": (ctypes.c_double, [ctypes.c_double]),
        "fdlbm_quartic_s_q": (ctypes.c_double, [ctypes.c_double]),
        "fdlbm_device_copy": (i32, [vp, vp, ctypes.c_size_t, vp]),
        "fdlbm_autotune": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dp]),
        "fdlbm_batch_workspace_bytes": (i32, [ctypes.POINTER(Instance), i32, i32, i32, ctypes.POINTER(ctypes.c_size_t),
                                              ctypes.POINTER(ctypes.c_size_t)]),
        "fdlbm_batch_create": (i32, [ctypes.POINTER(Instance), i32, i32, i32, vp, vp, vp, ctypes.c_size_t, vp,
                                     ctypes.POINTER(vp)]),
        "fdlbm_batch_set_state": (i32, [vp, i32, dp, dp, dp]),
        "fdlbm_batch_get_state": (i32, [vp, i32, dp, dp, dp]),
        "fdlbm_batch_step": (i32, [vp, i64, i32, i32]),
        "fdlbm_batch_step_per_instance": (i32, [vp, i64]),
        "fdlbm_batch_amplitudes": (i32, [vp, dp, ctypes.POINTER(ctypes.c_int32)]),
        "fdlbm_batch_step_count": (i64, [vp]),
        "fdlbm_batch_destroy": (None, [vp]),
        "fdlbm_batch_last_error": (ctypes.c_char_p, []),
        "fdlbm_batch_autotune": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int32), dp]),
        "fdlbm3d_workspace_bytes": (i32, [ctypes.POINTER(Params3D), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t)]),
        "fdlbm3d_create": (i32, [ctypes.POINTER(Params3D), vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "fdlbm3d_set_state": (i32, [vp, dp, dp, dp, dp]),
        "fdlbm3d_get_state": (i32, [vp, dp, dp, dp, dp]),
        "fdlbm3d_step": (i32, [vp, i64]),
        "fdlbm3d_diagnostics": (i32, [vp, ctypes.POINTER(Diag3D)]),
        "fdlbm3d_step_count": (i64, [vp]),
        "fdlbm3d_destroy": (None, [vp]),
        "fdlbm3d_last_error": (ctypes.c_char_p, []),
        "fdlbm3d_autotune": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _check(rc, what):
    if rc != FDLBM_OK:
        raise FdlbmError(rc, what)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------- C-named entry points ----

def make_params(nx, ny, scheme="fd", stencil=3, bc="periodic", dtype="f32", s_xx=1.0, s_e=1.0,
                s_q=1.0, s_eps=1.0, quartic=False, force=(0.0, 0.0), kernel="auto", tile_rows=0,
                check_every=0, lane_cols=0, wall_xi=0.5, disk=(0.0, 0.0, 0.0)):
    """disk = (cx, cy, R) with bc="disk": the curved no-slip wall of section 3-b."""
    return Params(int(nx), int(ny), SCHEME[scheme], int(stencil), BC[bc], DTYPE[dtype], float(s_xx),
                  float(s_e), float(s_q), float(s_eps), int(bool(quartic)), float(force[0]),
                  float(force[1]), KERNEL[kernel], int(tile_rows), int(check_every), int(lane_cols),
                  float(wall_xi), float(disk[0]), float(disk[1]), float(disk[2]))


def fdlbm_workspace_bytes(params):
    sb, cb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().fdlbm_workspace_bytes(ctypes.byref(params), ctypes.byref(sb), ctypes.byref(cb)),
           "fdlbm_workspace_bytes")
    return sb.value, cb.value


def fdlbm_create(params, state_a, state_b, scratch, scratch_bytes, stream):
    """Device pointers as ints; stream a hipStream_t handle as int (0 = default)."""
    ctx = ctypes.c_void_p()
    _check(load_library().fdlbm_create(ctypes.byref(params), state_a, state_b, scratch, scratch_bytes,
                                       stream or None, ctypes.byref(ctx)), "fdlbm_create")
    return ctx


def fdlbm_set_state(ctx, drho, jx, jy):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (drho, jx, jy)]
    _check(load_library().fdlbm_set_state(ctx, *[_dptr(v) for v in a]), "fdlbm_set_state")


def fdlbm_get_state(ctx, shape):
    out = [np.empty(shape, dtype=np.float64) for _ in range(3)]
    _check(load_library().fdlbm_get_state(ctx, *[_dptr(v) for v in out]), "fdlbm_get_state")
    return tuple(out)


def fdlbm_set_populations(ctx, df):
    a = np.ascontiguousarray(df, dtype=np.float64)
    _check(load_library().fdlbm_set_populations(ctx, _dptr(a)), "fdlbm_set_populations")


def fdlbm_get_populations(ctx, shape):
    out = np.empty((9,) + tuple(shape), dtype=np.float64)
    _check(load_library().fdlbm_get_populations(ctx, _dptr(out)), "fdlbm_get_populations")
    return out


def fdlbm_step(ctx, nsteps):
    _check(load_library().fdlbm_step(ctx, int(nsteps)), "fdlbm_step")


def mrt_step(ctx, nsteps):
    _check(load_library().mrt_step(ctx, int(nsteps)), "mrt_step")


def lwacm_step(ctx, nsteps):
    _check(load_library().lwacm_step(ctx, int(nsteps)), "lwacm_step")


def fdlbm_diagnostics(ctx):
    d = Diag()
    _check(load_library().fdlbm_diagnostics(ctx, ctypes.byref(d)), "fdlbm_diagnostics")
    return {f: getattr(d, f) for f, _ in Diag._fields_}


def fdlbm_diagnostics_static(params, state, out, j0x=0, j0y=0, stream=0):
    """Allocation-free diagnostics of the state in device buffer `state` (int pointer, the
    layout of `params`), written asynchronously as 8 doubles to device memory `out`; j0x, j0y
    optional device FP64 planes.  Nothing synchronises."""
    _check(load_library().fdlbm_diagnostics_static(ctypes.byref(params), state, j0x or None, j0y or None,
                                                   stream or None, out), "fdlbm_diagnostics_static")


def fdlbm_set_mode(ctx, j0x, j0y):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (j0x, j0y)]
    _check(load_library().fdlbm_set_mode(ctx, *[_dptr(v) for v in a]), "fdlbm_set_mode")


def fdlbm_mode_projection(ctx):
    out = ctypes.c_double()
    _check(load_library().fdlbm_mode_projection(ctx, ctypes.byref(out)), "fdlbm_mode_projection")
    return out.value


def fdlbm_step_count(ctx):
    return int(load_library().fdlbm_step_count(ctx))


def fdlbm_set_step_count(ctx, steps):
    _check(load_library().fdlbm_set_step_count(ctx, int(steps)), "fdlbm_set_step_count")


def fdlbm_destroy(ctx):
    load_library().fdlbm_destroy(ctx)


def fdlbm_rate_from_viscosity(nu):
    return float(load_library().fdlbm_rate_from_viscosity(float(nu)))


def fdlbm_quartic_s_q(s_xx):
    return float(load_library().fdlbm_quartic_s_q(float(s_xx)))


def fdlbm_autotune(ctx, reps=20):
    """Time the candidate tile shapes of this context's step kernel and keep the fastest.
    Returns (lane_cols, tile_rows, ms_per_step); the state does not advance."""
    cols, rows, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load_library().fdlbm_autotune(ctx, int(reps), ctypes.byref(cols), ctypes.byref(rows), ctypes.byref(ms)),
           "fdlbm_autotune")
    return cols.value, rows.value, ms.value


def fdlbm_device_copy(dst, src, nbytes, stream=0):
    """Streaming copy of nbytes between device pointers (ints) on a HIP stream handle."""
    _check(load_library().fdlbm_device_copy(dst, src, int(nbytes), stream or None), "fdlbm_device_copy")


# ----------------------------------------------------------------- convenience ----

@dataclass
class Buffers:
    state_a: object
    state_b: object
    scratch: object


class FdLbm:
    """One simulation: owns its torch device buffers and its library context.

    Keyword arguments follow ``fdlbm_params`` (see include/fdlbm.h); ``dtype`` is one of
    "f64", "f32", "f16" (FP16-stored deviations, FP32 arithmetic), "f16sr" (the same, new
    values rounded stochastically), ``bc`` "periodic",
    "walls" or "disk" (with ``disk=(cx, cy, R)``), ``scheme`` "fd", "mrt" or "lwacm",
    ``kernel`` "auto", "reference" or "sweep".
    """

    def __init__(self, nx, ny, device="cuda", stream=None, **kw):
        import torch

        load_library()
        self.nx, self.ny = int(nx), int(ny)
        self.params = make_params(nx, ny, **kw)
        self.scheme = kw.get("scheme", "fd")
        sb, cb = fdlbm_workspace_bytes(self.params)
        dev = torch.device(device)
        self._torch = torch
        self.buffers = Buffers(*(torch.empty(b, dtype=torch.uint8, device=dev) for b in (sb, sb, cb)))
        for t in (self.buffers.state_a, self.buffers.state_b, self.buffers.scratch):
            if t.data_ptr() % 256:
                raise RuntimeError("torch returned a device buffer that is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = fdlbm_create(self.params, self.buffers.state_a.data_ptr(), self.buffers.state_b.data_ptr(),
                                self.buffers.scratch.data_ptr(), cb, self.stream.cuda_stream)
        self.state_bytes, self.scratch_bytes = sb, cb

    # state
    def set_state(self, drho, jx, jy):
        fdlbm_set_state(self.ctx, drho, jx, jy)

    def get_state(self):
        return fdlbm_get_state(self.ctx, (self.ny, self.nx))

    def set_populations(self, df):
        fdlbm_set_populations(self.ctx, df)

    def get_populations(self):
        return fdlbm_get_populations(self.ctx, (self.ny, self.nx))

    # stepping
    def step(self, nsteps=1):
        if self.scheme == "mrt":
            mrt_step(self.ctx, nsteps)
        elif self.scheme == "lwacm":
            lwacm_step(self.ctx, nsteps)
        else:
            fdlbm_step(self.ctx, nsteps)

    @property
    def steps(self):
        return fdlbm_step_count(self.ctx)

    @steps.setter
    def steps(self, n):
        """Restore the step count (it seeds stochastic rounding; see fdlbm_set_step_count)."""
        fdlbm_set_step_count(self.ctx, n)

    def autotune(self, reps=20):
        """Pick the fastest tile shape for this grid (fdlbm_autotune); returns
        (lane_cols, tile_rows, ms_per_step)."""
        return fdlbm_autotune(self.ctx, reps)

    # diagnostics
    def diagnostics(self):
        return fdlbm_diagnostics(self.ctx)

    def set_mode(self, j0x, j0y):
        fdlbm_set_mode(self.ctx, j0x, j0y)

    def mode_projection(self):
        return fdlbm_mode_projection(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            fdlbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------- batches ----

def _instances(specs):
    arr = (Instance * len(specs))()
    for i, (nx, ny, s_xx, s_e) in enumerate(specs):
        arr[i] = Instance(int(nx), int(ny), float(s_xx), float(s_e))
    return arr


def fdlbm_batch_workspace_bytes(specs, dtype="f32", max_samples=0):
    arr = _instances(specs)
    sb, cb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().fdlbm_batch_workspace_bytes(arr, len(specs), DTYPE[dtype], int(max_samples), ctypes.byref(sb),
                                                      ctypes.byref(cb)), "fdlbm_batch_workspace_bytes")
    return sb.value, cb.value


class FdLbmBatch:
    """Many independent periodic FD-LBM grids (3-point differences) advanced together.

    specs: list of (nx, ny, s_xx, s_e); dtype "f64", "f32" or "f16" (stochastic rounding is
    for single grids only).  Uses its own HIP stream (default priority), which graph replay
    needs.
    """

    def __init__(self, specs, dtype="f32", max_samples=0, device="cuda"):
        import torch

        lib = load_library()
        self.specs = [tuple(x) for x in specs]
        self.count = len(self.specs)
        self.max_samples = int(max_samples)
        arr = _instances(self.specs)
        sb, cb = fdlbm_batch_workspace_bytes(self.specs, dtype, max_samples)
        dev = torch.device(device)
        self._bufs = [torch.empty(b, dtype=torch.uint8, device=dev) for b in (sb, sb, cb)]
        self.stream = torch.cuda.Stream(device=dev)
        self.ctx = ctypes.c_void_p()
        rc = lib.fdlbm_batch_create(arr, self.count, DTYPE[dtype], self.max_samples, self._bufs[0].data_ptr(),
                                    self._bufs[1].data_ptr(), self._bufs[2].data_ptr(), cb, self.stream.cuda_stream,
                                    ctypes.byref(self.ctx))
        if rc != FDLBM_OK:
            raise FdlbmError(rc, "fdlbm_batch_create: " + lib.fdlbm_batch_last_error().decode())
        self.state_bytes, self.scratch_bytes = sb, cb

    def _chk(self, rc, what):
        if rc != FDLBM_OK:
            raise FdlbmError(rc, what + ": " + load_library().fdlbm_batch_last_error().decode())

    def set_state(self, i, drho, jx, jy):
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (drho, jx, jy)]
        self._chk(load_library().fdlbm_batch_set_state(self.ctx, int(i), *[_dptr(v) for v in a]), "fdlbm_batch_set_state")

    def get_state(self, i):
        nx, ny = self.specs[i][0], self.specs[i][1]
        out = [np.empty((ny, nx)) for _ in range(3)]
        self._chk(load_library().fdlbm_batch_get_state(self.ctx, int(i), *[_dptr(v) for v in out]),
                  "fdlbm_batch_get_state")
        return tuple(out)

    def step(self, nsteps, sample_every=0, use_graph=True):
        self._chk(load_library().fdlbm_batch_step(self.ctx, int(nsteps), int(sample_every),
                                                  int(bool(use_graph and sample_every > 0))), "fdlbm_batch_step")

    def step_per_instance(self, nsteps):
        self._chk(load_library().fdlbm_batch_step_per_instance(self.ctx, int(nsteps)), "fdlbm_batch_step_per_instance")

    def autotune(self, reps=5):
        """Pick the fastest rows per wavefront for the one-launch step (fdlbm_batch_autotune);
        returns (rows, ms_per_step).  No step is taken."""
        rows, ms = ctypes.c_int32(), ctypes.c_double()
        self._chk(load_library().fdlbm_batch_autotune(self.ctx, int(reps), ctypes.byref(rows), ctypes.byref(ms)),
                  "fdlbm_batch_autotune")
        return rows.value, ms.value

    def amplitudes(self):
        """(count, nsamples) array of A(t) samples."""
        out = np.empty((self.count, max(self.max_samples, 1)))
        n = ctypes.c_int32()
        self._chk(load_library().fdlbm_batch_amplitudes(self.ctx, _dptr(out), ctypes.byref(n)), "fdlbm_batch_amplitudes")
        return out[:, :n.value].copy()

    @property
    def steps(self):
        return int(load_library().fdlbm_batch_step_count(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            load_library().fdlbm_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ D3Q19 (3D) ----

def make_params3d(nx, ny, nz, dtype="f32", s_nu=1.0, s_e=1.0, kernel="auto", tile_rows=0, tile_planes=0):
    if dtype not in ("f64", "f32"):
        raise ValueError("the D3Q19 step stores FP64 or FP32")
    return Params3D(int(nx), int(ny), int(nz), DTYPE[dtype], float(s_nu), float(s_e), KERNEL[kernel],
                    int(tile_rows), int(tile_planes))


def fdlbm3d_workspace_bytes(params):
    sb, cb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().fdlbm3d_workspace_bytes(ctypes.byref(params), ctypes.byref(sb), ctypes.byref(cb)),
           "fdlbm3d_workspace_bytes")
    return sb.value, cb.value


def fdlbm3d_create(params, state_a, state_b, scratch, scratch_bytes, stream):
    ctx = ctypes.c_void_p()
    _check(load_library().fdlbm3d_create(ctypes.byref(params), state_a, state_b, scratch, scratch_bytes, stream,
                                         ctypes.byref(ctx)), "fdlbm3d_create")
    return ctx


def fdlbm3d_set_state(ctx, drho, jx, jy, jz):
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (drho, jx, jy, jz)]
    _check(load_library().fdlbm3d_set_state(ctx, *(_dptr(x) for x in a)), "fdlbm3d_set_state")


def fdlbm3d_get_state(ctx, shape):
    out = [np.empty(shape, dtype=np.float64) for _ in range(4)]
    _check(load_library().fdlbm3d_get_state(ctx, *(_dptr(x) for x in out)), "fdlbm3d_get_state")
    return tuple(out)


def fdlbm3d_step(ctx, nsteps):
    _check(load_library().fdlbm3d_step(ctx, int(nsteps)), "fdlbm3d_step")


def fdlbm3d_diagnostics(ctx):
    d = Diag3D()
    _check(load_library().fdlbm3d_diagnostics(ctx, ctypes.byref(d)), "fdlbm3d_diagnostics")
    return {k: getattr(d, k) for k, _ in Diag3D._fields_}


def fdlbm3d_step_count(ctx):
    return int(load_library().fdlbm3d_step_count(ctx))


def fdlbm3d_destroy(ctx):
    load_library().fdlbm3d_destroy(ctx)


def fdlbm3d_last_error():
    return load_library().fdlbm3d_last_error().decode()


def fdlbm3d_autotune(ctx, reps=10):
    rows, planes, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load_library().fdlbm3d_autotune(ctx, int(reps), ctypes.byref(rows), ctypes.byref(planes),
                                           ctypes.byref(ms)), "fdlbm3d_autotune")
    return rows.value, planes.value, ms.value


class FdLbm3D:
    """One D3Q19 FD-LBM simulation on a periodic nx * ny * nz grid: owns its torch device
    buffers and its library context.  Keyword arguments follow ``fdlbm3d_params``
    (include/fdlbm3d.h): ``dtype`` "f64" or "f32", ``s_nu``, ``s_e``, ``kernel`` "auto",
    "reference" or "sweep", ``tile_rows`` (8, 12 or 16), ``tile_planes``.  Host arrays have shape
    (nz, ny, nx)."""

    def __init__(self, nx, ny, nz, device="cuda", stream=None, **kw):
        import torch

        load_library()
        self.shape = (int(nz), int(ny), int(nx))
        self.params = make_params3d(nx, ny, nz, **kw)
        sb, cb = fdlbm3d_workspace_bytes(self.params)
        dev = torch.device(device)
        self.buffers = Buffers(*(torch.empty(b, dtype=torch.uint8, device=dev) for b in (sb, sb, cb)))
        for t in (self.buffers.state_a, self.buffers.state_b, self.buffers.scratch):
            if t.data_ptr() % 256:
                raise RuntimeError("torch returned a device buffer that is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = fdlbm3d_create(self.params, self.buffers.state_a.data_ptr(), self.buffers.state_b.data_ptr(),
                                  self.buffers.scratch.data_ptr(), cb, self.stream.cuda_stream)
        self.state_bytes, self.scratch_bytes = sb, cb

    def set_state(self, drho, jx, jy, jz):
        fdlbm3d_set_state(self.ctx, drho, jx, jy, jz)

    def get_state(self):
        return fdlbm3d_get_state(self.ctx, self.shape)

    def step(self, nsteps=1):
        fdlbm3d_step(self.ctx, nsteps)

    @property
    def steps(self):
        return fdlbm3d_step_count(self.ctx)

    def diagnostics(self):
        return fdlbm3d_diagnostics(self.ctx)

    def autotune(self, reps=10):
        """Pick the fastest sweep tile shape for this grid (fdlbm3d_autotune); returns
        (tile_rows, tile_planes, ms_per_step)."""
        return fdlbm3d_autotune(self.ctx, reps)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            fdlbm3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
