"""FP64 oracle of the FD-LBM step on the D3Q19 lattice, and its linear symbol.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this module.

The Conclusion of the paper says the analysis of section 2 was also carried out for D3Q19
but prints no expression.  ``fd3d_oracle.c`` (loaded here) applies the construction of
section 2 to D3Q19: the polynomial moment basis of d'Humieres et al. (2002), second-order
equilibria, the six second-order moments relaxed with the defects of conservation theta
(eq. theta, expanded at rho close to 1 with v read as J, as section 2 does for D2Q9), every
other moment at equilibrium, 3-point differences, propagation by eq. 2.  Its header lists
the readings D1-D5.

``fd3d_symbol`` is a second, independent rendering of the same step, linearised about a
uniform state (rho = 1, J = V) for a plane wave exp(i k.x): the amplification matrix H(k)
of the state (drho, Jx, Jy, Jz), as in the von Neumann analysis of section 2.  It is written
from the same readings, not from the C code, and the tests check one against the other.

Array convention: float64 arrays of shape (nz, ny, nx), x fastest; the state is the deviation
from rest (drho = rho - 1, jx, jy, jz).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _c, _check, _dp, _load

_i32p = ctypes.POINTER(ctypes.c_int32)


def _lib():
    lib = _load()
    if not getattr(lib, "_d3q19_ready", False):
        i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        lib.oracle_fd3d_step.argtypes = [i32, i32, i32, dbl, dbl, _dp, _dp, _dp, _dp, i64]
        lib.oracle_fd3d_step.restype = i32
        lib.oracle_fd3d_theta.argtypes = [i32, i32, i32, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_fd3d_theta.restype = i32
        lib.oracle_d3q19_velocities.argtypes = [_i32p, _i32p, _i32p]
        lib.oracle_d3q19_moment_matrix.argtypes = [_dp]
        lib._d3q19_ready = True
    return lib


def velocities():
    """The oracle's velocity order, as three int arrays of 19 (cx, cy, cz)."""
    c = [np.empty(19, dtype=np.int32) for _ in range(3)]
    _lib().oracle_d3q19_velocities(*(a.ctypes.data_as(_i32p) for a in c))
    return tuple(c)


def moment_matrix():
    out = np.empty(361)
    _lib().oracle_d3q19_moment_matrix(out.ctypes.data_as(_dp))
    return out.reshape(19, 19)


def fd3d_run(drho, jx, jy, jz, nsteps, *, s_nu, s_e=1.0):
    """Advance the D3Q19 FD-LBM state by nsteps on a periodic grid; returns the new
    (drho, jx, jy, jz)."""
    f = [_c(np.array(a, dtype=np.float64, copy=True)) for a in (drho, jx, jy, jz)]
    nz, ny, nx = f[0][0].shape
    _check(_lib().oracle_fd3d_step(nx, ny, nz, float(s_e), float(s_nu), *(p for _, p in f), int(nsteps)),
           "fd3d_step")
    return tuple(a for a, _ in f)


def fd3d_theta(drho, jx, jy, jz):
    """The six defects theta (for e, 3p_xx, p_ww, p_xy, p_yz, p_xz) at every node, as the
    step evaluates them; shape (6, nz, ny, nx)."""
    f = [_c(a) for a in (drho, jx, jy, jz)]
    nz, ny, nx = f[0][0].shape
    out = np.empty((6, nz, ny, nx))
    _check(_lib().oracle_fd3d_theta(nx, ny, nz, *(p for _, p in f), out.ctypes.data_as(_dp)), "fd3d_theta")
    return out


def rate_from_viscosity(nu):
    """nu = (1/s - 1/2)/3, the same relation as section 1-a."""
    return 1.0 / (0.5 + 3.0 * nu)


# ----------------------------------------------------------------- linear symbol ----

def _lattice():
    c = [(0, 0, 0)]
    for a in range(3):
        for s in (1, -1):
            e = [0, 0, 0]
            e[a] = s
            c.append(tuple(e))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa, sb in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
            e = [0, 0, 0]
            e[a], e[b] = sa, sb
            c.append(tuple(e))
    c = np.array(c, dtype=float)
    c2 = np.sum(c * c, axis=1)
    w = np.where(c2 == 0, 1 / 3, np.where(c2 == 1, 1 / 18, 1 / 36))
    return c, w


def _basis(c):
    x, y, z = c.T
    c2 = x * x + y * y + z * z
    rows = {
        "rho": np.ones_like(x), "e": 19 * c2 - 30, "eps": (21 * c2 * c2 - 53 * c2 + 24) / 2,
        "jx": x, "qx": (5 * c2 - 9) * x, "jy": y, "qy": (5 * c2 - 9) * y, "jz": z, "qz": (5 * c2 - 9) * z,
        "pxx": 3 * x * x - c2, "pixx": (3 * c2 - 5) * (3 * x * x - c2), "pww": y * y - z * z,
        "piww": (3 * c2 - 5) * (y * y - z * z), "pxy": x * y, "pyz": y * z, "pxz": x * z,
        "mx": x * (y * y - z * z), "my": y * (z * z - x * x), "mz": z * (x * x - y * y),
    }
    names = list(rows)
    return names, np.array([rows[n] for n in names])


def fd3d_symbol(k, *, s_nu, s_e=1.0, V=(0.0, 0.0, 0.0)):
    """Amplification matrix H(k) (4 x 4 over drho, Jx, Jy, Jz) of one step for a plane wave
    exp(i k.x) of small amplitude on the uniform state rho = 1, J = V.

    Linearised pieces: a 3-point difference of a plane wave is i sin(k_a) times it; a product
    J_a J_b varies by V_a dJ_b + V_b dJ_a; the equilibrium moments vary by the derivative of
    the second-order polynomial at (1, V); the defects theta (readings D3, D4) vary by their
    terms linear in the wave; f* = M^{-1} m*; propagation multiplies population q by
    exp(-i k.c_q) before the moments rho and J are summed."""
    k = np.asarray(k, dtype=float)
    V = np.asarray(V, dtype=float)
    c, w = _lattice()
    names, M = _basis(c)
    Minv = M.T / np.sum(M * M, axis=1)
    s = 1j * np.sin(k)
    e = np.eye(4)
    dr, dJ = e[0], [e[1 + a] for a in range(3)]
    # equilibrium f^eq_q = w_q [rho + 3 c.J + 9/2 (c.J)^2/rho - 3/2 |J|^2/rho], its derivative at (1, V)
    cu = c @ V
    jac = np.zeros((19, 4))
    jac[:, 0] = w * (1 - 4.5 * cu * cu + 1.5 * (V @ V))
    for a in range(3):
        jac[:, 1 + a] = w * (3 * c[:, a] + 9 * cu * c[:, a] - 3 * V[a])
    dm = (M @ jac).astype(complex)
    # defects
    D = [sum(s[cc] * (V[a] * dJ[cc] + V[cc] * dJ[a]) for cc in range(3)) for a in range(3)]
    t = [[(s[a] * dJ[b] + s[b] * dJ[a]) / 3 - (V[a] * s[b] + V[b] * s[a]) * dr / 3 - V[a] * D[b] - V[b] * D[a]
          for b in range(3)] for a in range(3)]
    div = sum(s[a] * dJ[a] for a in range(3))
    tr = 2 / 3 * div - 2 / 3 * sum(V[a] * s[a] for a in range(3)) * dr - 2 * (V @ V) * div
    ce, cn = 1 - 1 / s_e, 1 - 1 / s_nu
    add = {"e": ce * 19 * tr, "pxx": cn * (2 * t[0][0] - t[1][1] - t[2][2]), "pww": cn * (t[1][1] - t[2][2]),
           "pxy": cn * t[0][1], "pyz": cn * t[1][2], "pxz": cn * t[0][2]}
    for n, v in add.items():
        dm[names.index(n)] += v
    df = Minv @ dm
    ph = np.exp(-1j * (c @ k))
    P = np.vstack([np.ones(19), c.T])
    return P @ (ph[:, None] * df)
