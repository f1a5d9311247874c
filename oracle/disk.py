"""FD-LBM (and LW-ACM) state inside a disk closed by a curved no-slip wall (section 3-b).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3-b gives the principle only: the nodes just outside the fluid carry a virtual-fluid
state, obtained by linear extrapolation with zero velocity on the wall, with an expression
that depends on where the wall cuts the link from the last fluid node (as in the
interpolated bounce-back of Bouzidi et al.).  Reading taken here, the curved counterpart of
the straight-wall ghost rows:

  * fluid nodes: distance r < R from the centre (cx, cy).  Ghost nodes: every other node
    within Chebyshev distance 3 of a fluid node (one propagation link plus the two-node
    reach of the 5-point differences).  Every remaining node is held at rest (zero
    deviation).
  * A ghost node at r = R + delta on the ray of unit vector n takes the state found at its
    mirror point c + (R - delta) n across the wall, velocity negated and density kept
    (the velocity then vanishes on the wall), by bilinear interpolation when the four
    nodes around the mirror point are fluid.
  * Otherwise (the mirror point lies in the last cell before the wall) the velocity runs
    linearly from zero on the wall to a sample at depth 3/2 inside, on the same ray:
    J_ghost = -(delta / (3/2)) J(c + (R - 3/2) n), density that of the sample.  The four
    nodes around that sample are always fluid, since they lie within sqrt(2) < 3/2 of it.

Each step first fills the ghost and rest nodes from the fluid, then advances the whole grid
with the periodic step.  The grid keeps at least 3 nodes between the fluid and its edges,
so no periodic image enters the update of a fluid node.

The decay rate of a Stokes mode (Tables 2 and 3) is measured from the projection
A(t) = sum_fluid J(t).J(0) / sum_fluid J(0).J(0) at two times: Gamma = -log(A(t2)/A(t1)) /
(t2 - t1), t1 = 0.3 / Gamma_0 (acoustic start-up gone), t2 = t1 + 1 / Gamma_0, with
Gamma_0 = nu k^2 the continuum rate.
"""
from __future__ import annotations

import math

import numpy as np

from . import fd_run, lwacm_run, rate_from_viscosity

SAMPLE_DEPTH = 1.5
GHOST_REACH = 3


def disk_ghost_rules(nx, ny, cx, cy, R):
    """Fluid mask and the rule of every ghost node, by the reading in the module docstring.

    Returns a dict: ``fluid`` (bool (ny, nx)), ``rest`` (bool (ny, nx): neither fluid nor
    ghost), and per ghost node the arrays ``j``, ``i`` (its row and column), ``j0``, ``i0``
    (lower-left node of the interpolation cell), ``wy``, ``wx`` (bilinear weights of the
    upper/right neighbours) and ``sj`` (factor on the interpolated momentum: -1 for the
    mirror, -delta/1.5 for the wall interpolation); the density factor is always 1."""
    fluid = np.zeros((ny, nx), dtype=bool)
    for j in range(ny):
        for i in range(nx):
            fluid[j, i] = math.hypot(i - cx, j - cy) < R
    fj, fi = np.nonzero(fluid)
    if fj.size == 0:
        raise ValueError("no fluid node in the disk")
    g = GHOST_REACH
    if fi.min() < g or fj.min() < g or fi.max() > nx - 1 - g or fj.max() > ny - 1 - g:
        raise ValueError("the disk and its ghost nodes must fit in the grid without wrapping")
    ghost = np.zeros_like(fluid)
    for j in range(ny):
        for i in range(nx):
            if not fluid[j, i]:
                ghost[j, i] = fluid[max(j - g, 0):j + g + 1, max(i - g, 0):i + g + 1].any()

    def cell(px, py):
        i0, j0 = math.floor(px), math.floor(py)
        ok = fluid[j0, i0] and fluid[j0, i0 + 1] and fluid[j0 + 1, i0] and fluid[j0 + 1, i0 + 1]
        return i0, j0, px - i0, py - j0, ok

    rows = []
    for j, i in zip(*np.nonzero(ghost)):
        r = math.hypot(i - cx, j - cy)
        ux, uy = (i - cx) / r, (j - cy) / r
        delta = r - R
        i0, j0, wx, wy, ok = cell(cx + (R - delta) * ux, cy + (R - delta) * uy)
        sj = -1.0
        if not ok:
            i0, j0, wx, wy, ok = cell(cx + (R - SAMPLE_DEPTH) * ux, cy + (R - SAMPLE_DEPTH) * uy)
            assert ok
            sj = -delta / SAMPLE_DEPTH
        rows.append((j, i, j0, i0, wy, wx, sj))
    cols = list(zip(*rows))
    out = {"fluid": fluid, "rest": ~fluid & ~ghost}
    for name, col, dt in zip(("j", "i", "j0", "i0", "wy", "wx", "sj"), cols,
                             (int, int, int, int, float, float, float)):
        out[name] = np.array(col, dtype=dt)
    return out


def _bilinear(a, rules):
    j0, i0, wy, wx = rules["j0"], rules["i0"], rules["wy"], rules["wx"]
    return ((1 - wy) * ((1 - wx) * a[j0, i0] + wx * a[j0, i0 + 1])
            + wy * ((1 - wx) * a[j0 + 1, i0] + wx * a[j0 + 1, i0 + 1]))


def disk_fill(drho, jx, jy, rules):
    """The state with its ghost nodes set from the fluid and its rest nodes zeroed."""
    out = []
    for a, factor in ((drho, None), (jx, rules["sj"]), (jy, rules["sj"])):
        b = np.array(a, dtype=np.float64, copy=True)
        b[rules["rest"]] = 0.0
        v = _bilinear(a, rules)
        b[rules["j"], rules["i"]] = v if factor is None else factor * v
        out.append(b)
    return tuple(out)


def disk_run(drho, jx, jy, nsteps, *, rules, scheme="fd", s_xx, s_e=1.0, stencil=3, fx=0.0, fy=0.0,
             on_step=None):
    """nsteps of (fill the ghost nodes, then one periodic step of the whole grid).
    scheme "fd": FD-LBM of section 2; "lwacm": the LW-ACM step of section 1-b (nu from
    s_xx).  on_step(t, state), if given, sees the state after t steps (t = 0..nsteps)."""
    state = tuple(np.array(a, dtype=np.float64, copy=True) for a in (drho, jx, jy))
    nu = (1.0 / s_xx - 0.5) / 3.0
    for t in range(nsteps):
        if on_step is not None:
            on_step(t, state)
        state = disk_fill(*state, rules)
        if scheme == "fd":
            state = fd_run(*state, 1, s_xx=s_xx, s_e=s_e, stencil=stencil, fx=fx, fy=fy)
        elif scheme == "lwacm":
            state = lwacm_run(*state, 1, nu=nu)
        else:
            raise ValueError(scheme)
    if on_step is not None:
        on_step(nsteps, state)
    return state


def decay_times(gamma0):
    """(t1, t2) of the two-time rate measurement for a mode of continuum rate gamma0."""
    t1 = int(round(0.3 / gamma0))
    return t1, t1 + int(round(1.0 / gamma0))


def disk_decay_rate(init, *, rules, nu, gamma0, **kw):
    """Measured decay rate of the mode started from init (the module docstring's two-time
    projection), FD-LBM with s_xx from nu unless given."""
    t1, t2 = decay_times(gamma0)
    j0x, j0y = np.where(rules["fluid"], init[1], 0.0), np.where(rules["fluid"], init[2], 0.0)
    den = float(np.sum(j0x * j0x + j0y * j0y))
    amp = {}

    def sample(t, state):
        if t in (t1, t2):
            amp[t] = float(np.sum(state[1] * j0x + state[2] * j0y)) / den

    kw.setdefault("s_xx", rate_from_viscosity(nu))
    disk_run(*init, t2, rules=rules, on_step=sample, **kw)
    return -math.log(amp[t2] / amp[t1]) / (t2 - t1)


# ------------------------------------------------------------------ MRT D2Q9 in the disk ----
#
# The lattice Boltzmann columns of Tables 2 and 3 (BGK, MRT with and without the quartic
# condition) close the disk with the linear interpolated bounce-back of Bouzidi, Firdaouss
# and Lallemand, which section 3-b cites for its wall treatment.  Reading taken here:
#   * fluid nodes r < R as for FD-LBM; every other node is solid and held at rest;
#   * a boundary link joins a fluid node x and a solid node x + e_i; the wall cuts it at
#     x + q e_i, 0 < q <= 1 (the root of |x + q e_i - c| = R);
#   * after the periodic stream-collide step of the whole grid, the population that re-enters
#     x from that link, along i' = -e_i, is
#         q <  1/2:  2q f*_i(x) + (1 - 2q) f*_i(x - e_i)
#         q >= 1/2:  f*_i(x) / (2q) + (2q - 1)/(2q) f*_i'(x)
#     (halfway bounce-back f*_i(x) at q = 1/2); where x - e_i is solid too (a chord shorter
#     than two links) the q < 1/2 case takes halfway bounce-back;
#   * every post-collision value needed is still in the streamed grid: f*_i(x) sits at the
#     solid node x + e_i, f*_i(x - e_i) at x itself, f*_i'(x) at x - e_i.

def disk_links(nx, ny, cx, cy, R):
    """Fluid mask and every boundary link (fluid node, direction i toward the wall, q), with
    the same grid-fit rule as disk_ghost_rules.  Returns a dict: ``fluid`` (bool (ny, nx)),
    ``j``, ``i``, ``k`` (direction 1..8 toward the wall), ``q``, ``back`` (whether x - e_k
    is fluid)."""
    rules = disk_ghost_rules(nx, ny, cx, cy, R)  # same fluid set and grid-fit checks
    fluid = rules["fluid"]
    from .matrix_form import E
    rows = []
    for j, i in zip(*np.nonzero(fluid)):
        for k in range(1, 9):
            ex, ey = E[k]
            if fluid[j + ey, i + ex]:
                continue
            # |p + q e - c|^2 = R^2 with p inside: the root q in (0, 1]
            px, py = i - cx, j - cy
            a = ex * ex + ey * ey
            b = 2 * (px * ex + py * ey)
            c = px * px + py * py - R * R
            q = (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)
            assert 0.0 < q <= 1.0 + 1e-12, q
            rows.append((j, i, k, min(q, 1.0), bool(fluid[j - ey, i - ex])))
    cols = list(zip(*rows))
    out = {"fluid": fluid}
    for name, col, dt in zip(("j", "i", "k", "q", "back"), cols, (int, int, int, float, bool)):
        out[name] = np.array(col, dtype=dt)
    return out


def interpolated_bounce_back(new, links):
    """Apply the wall to populations `new` (9, ny, nx) just streamed by a periodic step of
    the whole grid: every population re-entering a fluid node across a boundary link is
    replaced by the interpolated bounce-back value.  All reads are of streamed values that
    no replacement changes, so the links are independent of each other."""
    from .matrix_form import E
    opp = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
    j, i, k, q, back = links["j"], links["i"], links["k"], links["q"], links["back"]
    ex, ey = E[k, 0], E[k, 1]
    kb = opp[k]
    fi_x = new[k, j + ey, i + ex]          # f*_k(x), streamed into the solid node x + e_k
    fb_x = new[kb, j - ey, i - ex]         # f*_k'(x), streamed into x - e_k
    fi_back = new[k, j, i]                 # f*_k(x - e_k), streamed into x
    low = np.where(back, 2 * q * fi_x + (1 - 2 * q) * fi_back, fi_x)
    high = fi_x / (2 * q) + (2 * q - 1) / (2 * q) * fb_x
    out = np.array(new, copy=True)
    out[kb, j, i] = np.where(q < 0.5, low, high)
    return out


def mrt_disk_run(df, nsteps, *, links, s_xx, s_e=1.0, s_q=None, s_eps=1.0, fx=0.0, fy=0.0, on_step=None):
    """nsteps of the MRT D2Q9 step (eqs. 1-2) of the whole grid, then the interpolated
    bounce-back on the disk's boundary links, then every solid node set to rest.  df:
    population deviations (9, ny, nx); on_step(t, df) sees the populations after t steps."""
    from . import mrt_run, quartic_s_q
    if s_q is None:
        s_q = quartic_s_q(s_xx)
    solid = ~links["fluid"]
    d = np.array(df, dtype=np.float64, copy=True)
    d[:, solid] = 0.0
    for t in range(nsteps):
        if on_step is not None:
            on_step(t, d)
        d = mrt_run(d, 1, s_xx=s_xx, s_e=s_e, s_q=s_q, s_eps=s_eps, fx=fx, fy=fy)
        d = interpolated_bounce_back(d, links)
        d[:, solid] = 0.0
    if on_step is not None:
        on_step(nsteps, d)
    return d


def mrt_disk_decay_rate(init, *, links, nu, gamma0, **kw):
    """Measured decay rate of the mode started from f = f^eq(init) (the same two-time
    projection as disk_decay_rate), MRT with s_xx from nu unless given."""
    from . import mrt_init, mrt_moments
    t1, t2 = decay_times(gamma0)
    fluid = links["fluid"]
    j0x, j0y = np.where(fluid, init[1], 0.0), np.where(fluid, init[2], 0.0)
    den = float(np.sum(j0x * j0x + j0y * j0y))
    amp = {}

    def sample(t, d):
        if t in (t1, t2):
            _, jx, jy = mrt_moments(d)
            amp[t] = float(np.sum(jx * j0x + jy * j0y)) / den

    kw.setdefault("s_xx", rate_from_viscosity(nu))
    mrt_disk_run(mrt_init(*init), t2, links=links, on_step=sample, **kw)
    return -math.log(amp[t2] / amp[t1]) / (t2 - t1)
