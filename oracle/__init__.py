"""FP64 CPU oracle of the FD-LBM and MRT D2Q9 steps (Dubois, Lallemand, Obrecht, Tekitek).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the HIP library and
never imports it.

Contents
  * ``fdlbm_oracle.c`` (loaded here through ctypes): the node-by-node FP64 step of the
    FD-LBM scheme (section 2), of the LW-ACM scheme it starts from (section 1-b) and of
    the MRT D2Q9 scheme (section 1, eqs. 1-2), with the
    3-, 5- and 9-point finite differences of section 2, periodic or walls at a distance xi
    beyond the first and last rows (section 3-c, Fig. 6) and a Strang-split body force
    (section 1).
  * ``matrix_form``: a second, independent NumPy rendering of the same steps written as
    whole-array matrix products with ``numpy.linalg.inv`` and ``numpy.roll``.
  * ``symbol``: the linear amplification matrix H(k) of both schemes (von Neumann
    analysis of section 1-b, dispersion equation of section 2) and the transport
    coefficients extracted from its eigenvalues.
  * ``d3q19``: the FD-LBM step carried over to the D3Q19 lattice (``fd3d_oracle.c``), which
    the Conclusion says was analysed without printing it, and its linear symbol.
  * ``disk``: the curved no-slip wall of section 3-b around a disk (FD-LBM and LW-ACM:
    ghost nodes filled from the fluid before each periodic step; MRT D2Q9: interpolated
    bounce-back on the boundary links after it) and the decay-rate measurement of the
    Stokes modes of Tables 2 and 3.

Every part is pinned by tests/test_oracle_pins.py, tests/test_oracle_disk.py and
tests/test_oracle_d3q19.py; the
velocity-cubic term of theta_E (whose printed sign is read as a slip, reading R6) by the bulk
viscosity zeta (1 - 3V^2) in a mean flow that section 2 states.

Array convention: float64 arrays of shape (ny, nx), x fastest; the state is the deviation
from rest (drho = rho - 1, jx, jy); populations are (9, ny, nx) deviations f_k - w_k.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.oracle_fd_step.argtypes = [i32, i32, i32, i32, dbl, dbl, dbl, dbl, dbl, _dp, _dp, _dp, i64]
    lib.oracle_fd_step.restype = i32
    lib.oracle_mrt_step.argtypes = [i32, i32, i32, dbl, dbl, dbl, dbl, dbl, dbl, dbl, _dp, i64]
    lib.oracle_mrt_step.restype = i32
    lib.oracle_fd_theta.argtypes = [i32, i32, i32, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_fd_theta.restype = i32
    lib.oracle_lwacm_step.argtypes = [i32, i32, dbl, _dp, _dp, _dp, i64]
    lib.oracle_lwacm_step.restype = i32
    lib.oracle_mrt_init.argtypes = [i32, i32, _dp, _dp, _dp, _dp]
    lib.oracle_mrt_init.restype = i32
    lib.oracle_mrt_moments.argtypes = [i32, i32, _dp, _dp, _dp, _dp]
    lib.oracle_mrt_moments.restype = i32
    lib.oracle_fd_derivative.argtypes = [i32, i32, i32, i32, _dp, _dp]
    lib.oracle_fd_derivative.restype = i32
    lib.oracle_moment_matrix.argtypes = [_dp]
    lib.oracle_inverse_moment_matrix.argtypes = [_dp]
    lib.oracle_velocities.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_num_threads.argtypes = [i32]
    lib.oracle_num_threads.restype = i32
    _lib = lib
    return lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def num_threads(n=0):
    """Set (n > 0) and return the OpenMP thread count of the oracle."""
    return int(_load().oracle_num_threads(int(n)))


def moment_matrix():
    out = np.empty(81)
    _load().oracle_moment_matrix(out.ctypes.data_as(_dp))
    return out.reshape(9, 9)


def inverse_moment_matrix():
    out = np.empty(81)
    _load().oracle_inverse_moment_matrix(out.ctypes.data_as(_dp))
    return out.reshape(9, 9)


def velocities():
    ex = np.empty(9, dtype=np.int32)
    ey = np.empty(9, dtype=np.int32)
    _load().oracle_velocities(ex.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              ey.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return ex, ey


def rate_from_viscosity(nu):
    """Section 1-a: nu = (1/s - 1/2)/3  =>  s = 1/(1/2 + 3 nu)."""
    return 1.0 / (0.5 + 3.0 * nu)


def quartic_s_q(s_xx):
    """Section 3-b: (1/s_xx - 1/2)(1/s_q - 1/2) = 1/6 (isotropic hyperviscosity)."""
    return 1.0 / (0.5 + 1.0 / (6.0 * (1.0 / s_xx - 0.5)))


def derivative(field, stencil, axis):
    """Periodic finite-difference derivative of section 2 (axis 0 = x, 1 = y)."""
    f, fp = _c(field)
    ny, nx = f.shape
    out = np.empty_like(f)
    _check(_load().oracle_fd_derivative(nx, ny, int(stencil), int(axis), fp, out.ctypes.data_as(_dp)),
           "derivative")
    return out


def fd_run(drho, jx, jy, nsteps, *, s_xx, s_e=1.0, stencil=3, walls=False, xi=0.5, fx=0.0, fy=0.0):
    """Advance the FD-LBM state (section 2) by nsteps; returns new (drho, jx, jy).  With
    walls, they lie at distance xi beyond the first and last rows (0 < xi <= 1)."""
    r, rp = _c(np.array(drho, dtype=np.float64, copy=True))
    x, xp = _c(np.array(jx, dtype=np.float64, copy=True))
    y, yp = _c(np.array(jy, dtype=np.float64, copy=True))
    ny, nx = r.shape
    _check(_load().oracle_fd_step(nx, ny, int(stencil), int(bool(walls)), float(xi), float(s_e), float(s_xx),
                                  float(fx), float(fy), rp, xp, yp, int(nsteps)), "fd_step")
    return r, x, y


def fd_theta(drho, jx, jy, stencil=3):
    """The defects theta_E, theta_XX, theta_XY of section 2 at every node (periodic, the
    momentum J in place of v), as the FD-LBM step evaluates them."""
    r, rp = _c(drho)
    x, xp = _c(jx)
    y, yp = _c(jy)
    ny, nx = r.shape
    out = [np.empty((ny, nx)) for _ in range(3)]
    _check(_load().oracle_fd_theta(nx, ny, int(stencil), rp, xp, yp, *(o.ctypes.data_as(_dp) for o in out)),
           "fd_theta")
    return tuple(out)


def lwacm_run(drho, jx, jy, nsteps, *, nu):
    """Advance the LW-ACM state (section 1-b, Theta = 1 - 6 nu; periodic) by nsteps."""
    r, rp = _c(np.array(drho, dtype=np.float64, copy=True))
    x, xp = _c(np.array(jx, dtype=np.float64, copy=True))
    y, yp = _c(np.array(jy, dtype=np.float64, copy=True))
    ny, nx = r.shape
    _check(_load().oracle_lwacm_step(nx, ny, float(nu), rp, xp, yp, int(nsteps)), "lwacm_step")
    return r, x, y


def mrt_init(drho, jx, jy):
    """Populations f = f^eq(rho, J) = M^{-1} m^eq (deviations), shape (9, ny, nx)."""
    r, rp = _c(drho)
    x, xp = _c(jx)
    y, yp = _c(jy)
    ny, nx = r.shape
    df = np.empty((9, ny, nx))
    _check(_load().oracle_mrt_init(nx, ny, rp, xp, yp, df.ctypes.data_as(_dp)), "mrt_init")
    return df


def mrt_moments(df):
    d, dp = _c(df)
    _, ny, nx = d.shape
    r, x, y = np.empty((ny, nx)), np.empty((ny, nx)), np.empty((ny, nx))
    _check(_load().oracle_mrt_moments(nx, ny, dp, r.ctypes.data_as(_dp), x.ctypes.data_as(_dp),
                                      y.ctypes.data_as(_dp)), "mrt_moments")
    return r, x, y


def mrt_run(df, nsteps, *, s_xx, s_e=1.0, s_q=None, s_eps=1.0, walls=False, xi=0.5, fx=0.0, fy=0.0):
    """Advance MRT populations (eqs. 1-2) by nsteps; s_q defaults to the quartic value.  With
    walls, they lie at distance xi beyond the first and last rows (interpolated bounce-back)."""
    if s_q is None:
        s_q = quartic_s_q(s_xx)
    d, dp = _c(np.array(df, dtype=np.float64, copy=True))
    _, ny, nx = d.shape
    _check(_load().oracle_mrt_step(nx, ny, int(bool(walls)), float(xi), float(s_e), float(s_xx), float(s_q),
                                   float(s_eps), float(fx), float(fy), dp, int(nsteps)), "mrt_step")
    return d
