"""Second FP64 rendering of the FD-LBM and MRT D2Q9 steps, as whole-array matrix algebra.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It is written independently of
``fdlbm_oracle.c``: the moment matrix is built from the polynomial meaning of each moment
(section 1: density, mass flux, energy, stresses, energy flux, square of energy) instead
of being typed from the printed table, M^{-1} comes from ``numpy.linalg.inv``, finite
differences and propagation use ``numpy.roll``, and walls use explicit padding.  The
tests require the two oracles to agree to rounding, which guards each against slips of
transcription in the other.

Same conventions as the C oracle: fields (ny, nx), x fastest, deviations from rest.
Covered: the FD-LBM step (3-, 5-, 9-point differences, periodic or walls at any distance
xi, body force), the MRT step (periodic or walls with interpolated bounce-back) and the
LW-ACM step of section 1-b.
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


def _ghosts(rows, g, parity, xi):
    """Ghost rows at distances 1..g beyond a wall that lies xi beyond rows[0] (rows[m] is the
    m-th fluid row counted from the wall).  Sections 3-b and 3-c (reading R18): the ghost at
    distance d beyond the wall holds the value at its mirror point d inside the fluid, the
    velocity negated (parity -1; density parity +1), interpolated linearly between the fluid
    rows around that point; a mirror point between the wall and rows[0] takes the velocity
    interpolated between zero on the wall and rows[0], and the density of rows[0]."""
    out = []
    for dist in range(1, g + 1):
        ym = dist - 2 * xi  # ghost row at -dist, wall at -xi: mirror point at -xi + (dist - xi)
        if ym >= 0:
            s0 = int(np.floor(ym))
            t = ym - s0
            v = (1 - t) * rows[s0] + (t * rows[s0 + 1] if t > 0 else 0.0)
            out.append(parity * v)
        elif parity > 0:
            out.append(np.array(rows[0], copy=True))
        else:
            out.append(-((ym + xi) / xi) * rows[0])
    return out


def _pad_walls(a, g, parity, xi=0.5):
    """g ghost rows on each side for walls at distance xi beyond the first and last rows
    (xi = 1/2: the mirror about y = -1/2 and y = ny - 1/2)."""
    lo = _ghosts(a, g, parity, xi)[::-1]          # rows -g .. -1
    hi = _ghosts(a[::-1], g, parity, xi)          # rows ny .. ny + g - 1
    return np.concatenate([np.array(lo), a, np.array(hi)], axis=0)


def fd_step(drho, jx, jy, *, s_xx, s_e=1.0, stencil=3, walls=False, xi=0.5, fx=0.0, fy=0.0):
    """One FD-LBM step (section 2) on whole arrays; walls at distance xi beyond the first and
    last rows."""
    g = 3 if walls else 0
    if walls:
        r = _pad_walls(drho, g, +1.0, xi)
        vx = _pad_walls(jx, g, -1.0, xi) + 0.5 * fx
        vy = _pad_walls(jy, g, -1.0, xi) + 0.5 * fy
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


def mrt_step(df, *, s_xx, s_e=1.0, s_q, s_eps=1.0, walls=False, xi=0.5, fx=0.0, fy=0.0):
    """One MRT step (eqs. 1-2) on whole arrays.  Walls at distance xi beyond the first and
    last rows: the population that would come from beyond a wall is the linear interpolated
    bounce-back of Bouzidi, Firdaouss and Lallemand of the one that left toward it, with the
    wall cutting the link at q = xi (halfway bounce-back at 1/2)."""
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
        q = xi
        for k, (ex, ey) in enumerate(E):
            if ey == 0:
                continue
            row = 0 if ey == 1 else -1       # the fluid row next to the wall it came through
            i = opp[k]                       # the population that left toward that wall
            out_i = fstar[i][row]
            if q < 0.5:
                # f*_i at x - e_i, the node one row further inside
                behind = _shift(fstar[i], -E[i][0], -E[i][1])[row]
                new[k][row] = 2 * q * out_i + (1 - 2 * q) * behind
            else:
                new[k][row] = out_i / (2 * q) + (2 * q - 1) / (2 * q) * fstar[k][row]
    return new


def mrt_run(df, nsteps, **kw):
    d = np.array(df, dtype=float)
    for _ in range(nsteps):
        d = mrt_step(d, **kw)
    return d


def lwacm_step(drho, jx, jy, *, nu):
    """One LW-ACM step (section 1-b) on whole periodic arrays: f*_k(x) = f^eq_k(x) +
    Theta (f^eo_k(x + e_k) - f^eo_k(x)), Theta = 1 - 6 nu, with f^eo the part of the
    equilibrium odd in J (its J and q moments), then f_k(x + e_k) = f*_k(x)."""
    theta = 1.0 - 6.0 * nu
    feq = np.einsum("kl,lyx->kyx", MINV, equilibrium_moments(drho, jx, jy))
    z = np.zeros_like(jx)
    feo = np.einsum("kl,lyx->kyx", MINV, np.stack([z, jx, jy, z, z, z, -jx, -jy, z]))
    new = np.empty_like(feq)
    for k, (ex, ey) in enumerate(E):
        fstar = feq[k] + theta * (_shift(feo[k], ex, ey) - feo[k])
        new[k] = _shift(fstar, -ex, -ey)
    m = np.einsum("lk,kyx->lyx", M[:3], new)
    return m[0], m[1], m[2]


def lwacm_run(drho, jx, jy, nsteps, **kw):
    s = (np.array(drho, dtype=float), np.array(jx, dtype=float), np.array(jy, dtype=float))
    for _ in range(nsteps):
        s = lwacm_step(*s, **kw)
    return s


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
