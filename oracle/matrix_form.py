"""Second FP64 rendering of the FD-LBM and MRT D2Q9 steps, as whole-array matrix algebra.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It is written independently of
``fdlbm_oracle.c``: the moment matrix is built from the polynomial meaning of each moment
(section 1: density, mass flux, energy, stresses, energy flux, square of energy) instead
of being typed from the printed table, M^{-1} comes from ``numpy.linalg.inv``, finite
differences and propagation use ``numpy.roll``, and walls use explicit padding.  The
tests require the two oracles to agree to rounding, which guards each against slips of
transcription in the other.

Same conventions as the C oracle: fields (ny, nx), x fastest, deviations from rest.
"""
from __future__ import annotations

import numpy as np

# Section 1 velocity set, ordered so that q_x, q_y, XX, XY rows read as printed.
E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])


def moment_matrix_from_polynomials():
    """Rows: 1, e_x, e_y, 3|e|^2-4, e_x^2-e_y^2, e_x e_y, (3|e|^2-5)e_x, (3|e|^2-5)e_y,
    (9|e|^4-21|e|^2+8)/2 evaluated on the nine velocities."""
    ex, ey = E[:, 0].astype(float), E[:, 1].astype(float)
    e2 = ex * ex + ey * ey
    rows = [np.ones(9), ex, ey, 3 * e2 - 4, ex * ex - ey * ey, ex * ey, (3 * e2 - 5) * ex,
            (3 * e2 - 5) * ey, (9 * e2 * e2 - 21 * e2 + 8) / 2]
    return np.array(rows)


M = moment_matrix_from_polynomials()
MINV = np.linalg.inv(M)

# finite-difference stencils of section 2 as (dx, dy, weight) lists for d/dx;
# d/dy uses the same list with dx and dy exchanged.
STENCILS = {
    3: [(1, 0, 0.5), (-1, 0, -0.5)],
    5: [(1, 0, 0.75), (-1, 0, -0.75), (2, 0, -0.125), (-2, 0, 0.125)],
    9: [(1, 0, 1.0), (-1, 0, -1.0), (1, 1, -0.25), (-1, 1, 0.25), (-1, -1, 0.25), (1, -1, -0.25)],
}


def _shift(a, dx, dy):
    """value at (x + dx, y + dy) for every node (periodic in both directions of the array)."""
    return np.roll(a, shift=(-dy, -dx), axis=(0, 1))


def ddx(a, stencil):
    return sum(w * _shift(a, dx, dy) for dx, dy, w in STENCILS[stencil])


def ddy(a, stencil):
    return sum(w * _shift(a, dy, dx) for dx, dy, w in STENCILS[stencil])


def _pad_walls(a, g, parity):
    """g ghost rows on each side; mirror about y=-1/2 and y=ny-1/2 with the given parity."""
    lo = parity * a[:g][::-1]
    hi = parity * a[-g:][::-1]
    return np.concatenate([lo, a, hi], axis=0)


def fd_step(drho, jx, jy, *, s_xx, s_e=1.0, stencil=3, walls=False, fx=0.0, fy=0.0):
    """One FD-LBM step (section 2) on whole arrays."""
    g = 3 if walls else 0
    if walls:
        r = _pad_walls(drho, g, +1.0)
        vx = _pad_walls(jx, g, -1.0) + 0.5 * fx
        vy = _pad_walls(jy, g, -1.0) + 0.5 * fy
    else:
        r, vx, vy = drho, jx + 0.5 * fx, jy + 0.5 * fy
    rho = 1.0 + r
    dxr, dyr = ddx(r, stencil), ddy(r, stencil)
    a, b = ddx(vx, stencil), ddy(vy, stencil)
    c, d = ddx(vy, stencil), ddy(vx, stencil)
    P, Q, R = vx * vx, vy * vy, vx * vy
    Px, Qy, Rx, Ry = ddx(P, stencil), ddy(Q, stencil), ddx(R, stencil), ddy(R, stencil)
    th_e = (2 - 6 * (P + Q)) * (a + b) - 2 * (vx * dxr + vy * dyr)
    th_xx = 2 / 3 * (a - b) - 2 / 3 * (vx * dxr - vy * dyr) - 2 * (vx * (Px + Ry) - vy * (Rx + Qy))
    th_xy = 1 / 3 * (c + d) - 1 / 3 * (vx * dyr + vy * dxr) - vx * (Rx + Qy) - vy * (Px + Ry)
    K = (P + Q) / rho
    dm = np.stack([r, vx + 0.5 * fx, vy + 0.5 * fy,
                   -2 * r + 3 * K + (1 - 1 / s_e) * th_e,
                   (P - Q) / rho + (1 - 1 / s_xx) * th_xx,
                   R / rho + (1 - 1 / s_xx) * th_xy,
                   -vx, -vy, r - 3 * K])
    fstar = np.einsum("kl,lyx->kyx", MINV, dm)
    new = np.empty_like(fstar)
    for k, (ex, ey) in enumerate(E):
        new[k] = _shift(fstar[k], -ex, -ey)  # f_new(x) = f*(x - e_k)
    if walls:
        new = new[:, g:-g]
    m = np.einsum("lk,kyx->lyx", M[:3], new)
    return m[0], m[1], m[2]


def fd_run(drho, jx, jy, nsteps, **kw):
    s = (np.array(drho, dtype=float), np.array(jx, dtype=float), np.array(jy, dtype=float))
    for _ in range(nsteps):
        s = fd_step(*s, **kw)
    return s


def equilibrium_moments(drho, jx, jy):
    rho = 1.0 + drho
    K = (jx * jx + jy * jy) / rho
    return np.stack([drho, jx, jy, -2 * drho + 3 * K, (jx * jx - jy * jy) / rho, jx * jy / rho,
                     -jx, -jy, drho - 3 * K])


def mrt_init(drho, jx, jy):
    return np.einsum("kl,lyx->kyx", MINV, equilibrium_moments(drho, jx, jy))


def mrt_step(df, *, s_xx, s_e=1.0, s_q, s_eps=1.0, walls=False, fx=0.0, fy=0.0):
    """One MRT step (eqs. 1-2) on whole arrays; halfway bounce-back on walls."""
    m = np.einsum("lk,kyx->lyx", M, df)
    meq = equilibrium_moments(m[0], m[1] + 0.5 * fx, m[2] + 0.5 * fy)
    s = np.array([0, 0, 0, s_e, s_xx, s_xx, s_q, s_q, s_eps])[:, None, None]
    ms = m + s * (meq - m)
    ms[1] = m[1] + fx
    ms[2] = m[2] + fy
    fstar = np.einsum("kl,lyx->kyx", MINV, ms)
    new = np.empty_like(fstar)
    for k, (ex, ey) in enumerate(E):
        new[k] = _shift(fstar[k], -ex, -ey)
    if walls:
        opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
        for k, (ex, ey) in enumerate(E):
            if ey == 1:  # would have come from beyond the lower wall
                new[k][0] = fstar[opp[k]][0]
            if ey == -1:
                new[k][-1] = fstar[opp[k]][-1]
    return new


def mrt_run(df, nsteps, **kw):
    d = np.array(df, dtype=float)
    for _ in range(nsteps):
        d = mrt_step(d, **kw)
    return d


def mrt_moments(df):
    m = np.einsum("lk,kyx->lyx", M[:3], df)
    return m[0], m[1], m[2]


def textbook_equilibrium(rho, ux_times_rho, uy_times_rho):
    """Polynomial D2Q9 equilibrium f_k = w_k [rho + 3 e.J + 9/2 (e.J)^2/rho - 3/2 |J|^2/rho]
    with w = 4/9, 1/9 (axes), 1/36 (diagonals) -- the textbook form, for cross-checks."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    jx, jy = ux_times_rho, uy_times_rho
    out = []
    for k, (ex, ey) in enumerate(E):
        ej = ex * jx + ey * jy
        out.append(w[k] * (rho + 3 * ej + 4.5 * ej * ej / rho - 1.5 * (jx * jx + jy * jy) / rho))
    return np.stack(out)
