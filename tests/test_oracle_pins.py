"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values printed in the
paper (Table 1, the quartic rate of section 3-b), closed forms of sections 1-a and 2
(transport coefficients, Galilean factor, hyperviscosity), exact invariants (mass and
momentum conservation, fixed points), a special case that reduces to the textbook BGK
scheme, the independently written linear symbol, and a second independent rendering of
the same steps.  No GPU is used.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import matrix_form as MF
from oracle import symbol as S

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fourier_coeff(field, mx, my):
    ny, nx = field.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.sum(field * np.exp(-2j * np.pi * (mx * x / nx + my * y / ny)))


# ---------------------------------------------------------------- section 1: moments ----

def test_velocity_set_is_d2q9():
    ex, ey = O.velocities()
    assert sorted(zip(ex.tolist(), ey.tolist())) == sorted((a, b) for a in (-1, 0, 1) for b in (-1, 0, 1))
    assert (ex[0], ey[0]) == (0, 0)


def test_moment_matrix_rows_are_the_physical_moments():
    """Section 1 names the rows: density, mass fluxes, energy, stresses, energy fluxes,
    square of energy.  As polynomials of the velocity e they are 1, e_x, e_y, 3|e|^2-4,
    e_x^2-e_y^2, e_x e_y, (3|e|^2-5)e, (9|e|^4-21|e|^2+8)/2; the printed energy, stress,
    energy-flux and eps rows are exactly these, which fixes the order of the velocities."""
    M = O.moment_matrix()
    ex, ey = (v.astype(float) for v in O.velocities())
    e2 = ex * ex + ey * ey
    expect = np.array([np.ones(9), ex, ey, 3 * e2 - 4, ex * ex - ey * ey, ex * ey,
                       (3 * e2 - 5) * ex, (3 * e2 - 5) * ey, (9 * e2 * e2 - 21 * e2 + 8) / 2])
    assert np.array_equal(M, expect)
    # rows printed in the section-1 table that carry no sign ambiguity
    assert M[3].tolist() == [-4, -1, -1, -1, -1, 2, 2, 2, 2]
    assert M[4].tolist() == [0, 1, -1, 1, -1, 0, 0, 0, 0]
    assert M[5].tolist() == [0, 0, 0, 0, 0, 1, -1, 1, -1]
    assert M[6].tolist() == [0, -2, 0, 2, 0, 1, -1, -1, 1]
    assert M[7].tolist() == [0, 0, -2, 0, 2, 1, 1, -1, -1]
    assert M[8].tolist() == [4, -2, -2, -2, -2, 1, 1, 1, 1]


def test_moment_matrix_is_orthogonal_and_inverse_is_exact():
    M = O.moment_matrix()
    assert np.array_equal(M @ M.T, np.diag([9.0, 6, 6, 36, 4, 4, 12, 12, 36]))
    assert np.allclose(O.inverse_moment_matrix() @ M, np.eye(9), atol=1e-15, rtol=0)
    assert np.allclose(O.inverse_moment_matrix(), np.linalg.inv(M), atol=1e-15, rtol=0)


def test_equilibrium_populations_are_the_textbook_polynomial():
    """M^{-1} m^eq with the section 1-a equilibria is the usual D2Q9 polynomial
    w_k [rho + 3 e.J + 9/2 (e.J)^2/rho - 3/2 |J|^2/rho]."""
    w = O.inverse_moment_matrix() @ np.array([1.0, 0, 0, -2, 0, 0, 0, 0, 1])
    assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-16, rtol=0)
    r, x, y = W.random_state(7, 5, seed=11, amp=0.05)
    df = O.mrt_init(r, x, y)
    f = df + w[:, None, None]
    ex, ey = O.velocities()
    wt = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rho = 1.0 + r
    for k in range(9):
        ej = ex[k] * x + ey[k] * y
        fk = wt[k] * (rho + 3 * ej + 4.5 * ej * ej / rho - 1.5 * (x * x + y * y) / rho)
        assert np.max(np.abs(f[k] - fk)) < 2e-16


# ------------------------------------------------- section 2: finite differences ----

@pytest.mark.parametrize("stencil", [3, 5, 9])
def test_finite_differences_exact_on_quadratics(stencil):
    n = 16
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    f = 0.3 + 0.7 * x - 1.1 * y + 0.05 * x * x - 0.02 * y * y + 0.03 * x * y
    dfx = 0.7 + 0.1 * x + 0.03 * y
    dfy = -1.1 - 0.04 * y + 0.03 * x
    inner = (slice(3, n - 3), slice(3, n - 3))
    gx, gy = O.derivative(f, stencil, 0), O.derivative(f, stencil, 1)
    assert np.max(np.abs(gx[inner] - dfx[inner])) < 1e-13
    assert np.max(np.abs(gy[inner] - dfy[inner])) < 1e-13


@pytest.mark.parametrize("stencil,err", [(3, 1.0), (5, -0.5), (9, 1.0)])
def test_finite_difference_error_on_cubics(stencil, err):
    """Section 2 leading errors: 3 points +h^2 f'''/6, 5 points -h^2 f'''/12 (so the
    5-point formula is second order by design); the 9-point formula reduces to the
    3-point one on a function of x alone.  With f = x^3 (f''' = 6) the errors are
    +1, -1/2 and +1 exactly; the same holds along y."""
    n = 16
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    inner = (slice(3, n - 3), slice(3, n - 3))
    gx = O.derivative(x ** 3, stencil, 0)
    gy = O.derivative(y ** 3, stencil, 1)
    assert np.max(np.abs(gx[inner] - (3 * x * x + err)[inner])) < 1e-11
    assert np.max(np.abs(gy[inner] - (3 * y * y + err)[inner])) < 1e-11


# ----------------------------------------------------- invariants of both schemes ----

@pytest.mark.parametrize("scheme", ["fd3", "fd5", "fd9", "mrt"])
def test_uniform_states_are_fixed_points(scheme):
    shape = (6, 7)
    r, x, y = (np.full(shape, v) for v in (0.01, 0.03, -0.02))
    if scheme == "mrt":
        out = O.mrt_moments(O.mrt_run(O.mrt_init(r, x, y), 10, s_xx=1.6, s_e=1.3, s_q=1.1, s_eps=1.2))
    else:
        out = O.fd_run(r, x, y, 10, s_xx=1.6, s_e=1.3, stencil=int(scheme[2]))
    for a, b in zip(out, (r, x, y)):
        assert np.max(np.abs(a - b)) < 1e-16


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_mass_and_momentum_conserved_on_periodic_grids(scheme):
    """rho and J are the conserved moments (section 1) and propagation permutes the
    populations (eq. 2): totals are invariant; a uniform force adds exactly F per node and
    per step to the total momentum (Strang splitting, J* = J + F)."""
    r, x, y = W.random_state(24, 20, seed=3, amp=0.02)
    n, steps = r.size, 200
    for fx, fy in ((0.0, 0.0), (1e-5, -3e-6)):
        if scheme == "mrt":
            out = O.mrt_moments(O.mrt_run(O.mrt_init(r, x, y), steps, s_xx=1.5, s_q=1.2, fx=fx, fy=fy))
        else:
            out = O.fd_run(r, x, y, steps, s_xx=1.5, stencil=int(scheme[2]), fx=fx, fy=fy)
        assert abs(out[0].sum() - r.sum()) < 1e-13
        assert abs(out[1].sum() - x.sum() - steps * n * fx) < 1e-12
        assert abs(out[2].sum() - y.sum() - steps * n * fy) < 1e-12


# ------------------------------------------------------------- two oracles agree ----

@pytest.mark.parametrize("stencil", [3, 5, 9])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("force", [0.0, 2e-4])
def test_c_oracle_equals_matrix_form(stencil, walls, force):
    r, x, y = W.random_state(13, 11, seed=5, amp=0.03)
    kw = dict(s_xx=1.7, s_e=1.25, stencil=stencil, walls=walls, fx=force, fy=-0.5 * force)
    a = O.fd_run(r, x, y, 8, **kw)
    b = MF.fd_run(r, x, y, 8, **kw)
    for u, v in zip(a, b):
        assert np.max(np.abs(u - v)) < 1e-16


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("xi", [0.15, 0.35, 0.5, 0.8, 1.0])
def test_c_oracle_equals_matrix_form_walls_at_any_distance(stencil, xi):
    """The ghost rows of walls at distance xi (reading R18), written independently in both
    renderings (the C one row by row from a rule table, the NumPy one from the mirror point
    of each ghost), give the same steps."""
    r, x, y = W.random_state(9, 10, seed=15, amp=0.03)
    kw = dict(s_xx=1.4, s_e=1.2, stencil=stencil, walls=True, xi=xi, fx=3e-4, fy=-1e-4)
    a = O.fd_run(r, x, y, 8, **kw)
    b = MF.fd_run(r, x, y, 8, **kw)
    for u, v in zip(a, b):
        assert np.max(np.abs(u - v)) < 1e-16


@pytest.mark.parametrize("walls,xi", [(False, 0.5), (True, 0.5), (True, 0.2), (True, 0.7), (True, 1.0)])
def test_mrt_c_oracle_equals_matrix_form(walls, xi):
    r, x, y = W.random_state(13, 11, seed=6, amp=0.03)
    df = O.mrt_init(r, x, y)
    assert np.max(np.abs(df - MF.mrt_init(r, x, y))) < 1e-17
    kw = dict(s_xx=1.7, s_e=1.25, s_q=1.1, s_eps=1.35, walls=walls, xi=xi, fx=1e-4, fy=2e-5)
    a = O.mrt_run(df, 8, **kw)
    b = MF.mrt_run(df, 8, **kw)
    assert np.max(np.abs(a - b)) < 1e-16


@pytest.mark.parametrize("nu", [0.02, 1 / 6, 0.1])
def test_lwacm_c_oracle_equals_matrix_form(nu):
    r, x, y = W.random_state(13, 11, seed=7, amp=0.03)
    a = O.lwacm_run(r, x, y, 8, nu=nu)
    b = MF.lwacm_run(r, x, y, 8, nu=nu)
    for u, v in zip(a, b):
        assert np.max(np.abs(u - v)) < 1e-16


# ----------------------------------------------- exact special case: BGK, tau = 1 ----

def test_unit_rates_reduce_to_textbook_bgk():
    """With every rate equal to 1 the post-collision populations are the equilibrium ones
    for both schemes (the theta terms carry the factor 1 - 1/s = 0): FD-LBM (3 or 5 points)
    and MRT must both equal textbook BGK with tau = 1, f(x, t+1) = f^eq(x - e_k, t)."""
    r, x, y = W.random_state(10, 9, seed=8, amp=0.03)
    ex, ey = O.velocities()
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    br, bx, by = r.copy(), x.copy(), y.copy()
    for _ in range(20):
        rho = 1.0 + br
        nr, nx_, ny_ = np.zeros_like(br), np.zeros_like(br), np.zeros_like(br)
        for k in range(9):
            ej = ex[k] * bx + ey[k] * by
            fk = w[k] * (rho + 3 * ej + 4.5 * ej * ej / rho - 1.5 * (bx * bx + by * by) / rho) - w[k]
            fk = np.roll(fk, shift=(ey[k], ex[k]), axis=(0, 1))
            nr += fk
            nx_ += ex[k] * fk
            ny_ += ey[k] * fk
        br, bx, by = nr, nx_, ny_
    for stencil in (3, 5):
        out = O.fd_run(r, x, y, 20, s_xx=1.0, s_e=1.0, stencil=stencil)
        for u, v in zip(out, (br, bx, by)):
            assert np.max(np.abs(u - v)) < 1e-15
    out = O.mrt_moments(O.mrt_run(O.mrt_init(r, x, y), 20, s_xx=1.0, s_e=1.0, s_q=1.0, s_eps=1.0))
    for u, v in zip(out, (br, bx, by)):
        assert np.max(np.abs(u - v)) < 1e-15


# --------------------------------------------------- linear symbol vs the paper ----

def test_symbol_reproduces_table1():
    g = json.load(open(os.path.join(GOLD, "table1_hyperviscosity.json")))
    for stencil, vals in g["nu2"].items():
        for ang, printed in zip(g["angles_deg"], vals):
            _, nu2 = S.hyperviscosity(math.radians(ang), s_xx=g["s_xx"], s_e=1.0, stencil=int(stencil))
            digits = len(repr(printed).split(".")[1])
            assert abs(nu2 - printed) <= 0.5 * 10.0 ** (-digits) + 1e-7, (stencil, ang, nu2, printed)


@pytest.mark.parametrize("s_xx", [1.2, 1.5, 1.85])
@pytest.mark.parametrize("s_e", [1.0, 1.4])
def test_symbol_transport_coefficients(s_xx, s_e):
    """Section 1-a / section 2: nu = (1/s_xx - 1/2)/3, c_s = 1/sqrt(3), and the sound
    root damps as (nu + zeta)/2 k^2 with zeta = (1/s_e - 1/2)/3."""
    nu, zeta = (1 / s_xx - 0.5) / 3, (1 / s_e - 0.5) / 3
    for stencil in (3, 5):
        nu0, _ = S.hyperviscosity(0.3, s_xx=s_xx, s_e=s_e, stencil=stencil)
        assert abs(nu0 - nu) < 1e-9
        k = 1e-3
        gs = S.sound_gammas(k * math.cos(0.4), k * math.sin(0.4), s_xx=s_xx, s_e=s_e, stencil=stencil)
        assert len(gs) == 2
        for g in gs:
            assert abs(abs(g.imag) / k - 1 / math.sqrt(3)) < 1e-6
            assert abs(g.real / k ** 2 - (nu + zeta) / 2) < 1e-5
    g = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    assert abs(1 / math.sqrt(3) - g["c_s"]) < 1e-15


@pytest.mark.parametrize("s_xx", [1.85, 1.5, 1.2])
def test_hyperviscosity_closed_forms(s_xx):
    """Section 2 closed forms, with the angular term entering with a plus sign
    (the printed minus contradicts Table 1: at 45 degrees it would give 0.0558 for the
    3-point stencil instead of the tabulated 0.01867), and the 9-point form written with
    the prefactors that reduce to the 3-point one on the x axis."""
    s = 1 / s_xx - 0.5
    for deg in (0.0, 26.6, 30.0, 45.0):
        c2 = math.cos(math.radians(deg)) ** 2
        ang = c2 - c2 * c2
        forms = {3: (2 * s - 3) * (2 * s - 1) / 72 + (8 * s - 3) / 36 * ang,
                 5: s * (2 * s - 1) / 36 + s / 18 * ang,
                 9: (2 * s - 3) * (2 * s - 1) / 72 + (20 * s - 9) / 36 * ang}
        for stencil, val in forms.items():
            _, nu2 = S.hyperviscosity(math.radians(deg), s_xx=s_xx, stencil=stencil)
            assert abs(nu2 - val) < 2e-6, (stencil, deg, nu2, val)


def test_quartic_condition_and_optimized_viscosity():
    """Section 3-b: (1/s_xx - 1/2)(1/s_q - 1/2) = 1/6 makes the D2Q9 hyperviscosity
    isotropic; at nu = 1/sqrt(108) it gives s_q = 0.9282 (printed) and a vanishing
    hyperviscosity, while s_q = 1.3 (the non-optimised run) is anisotropic."""
    g = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    nu = 1 / math.sqrt(108)
    assert abs(nu - g["quartic_nu"]) < 1e-15
    s_xx = O.rate_from_viscosity(nu)
    s_q = O.quartic_s_q(s_xx)
    assert abs(s_q - g["quartic_s_q_printed"]) < 0.5e-4
    assert abs((1 / s_xx - 0.5) * (1 / s_q - 0.5) - 1 / 6) < 1e-14
    angles = [0.0, math.radians(26.6), math.pi / 4]
    nu2 = [S.hyperviscosity(a, "mrt", s_xx=s_xx, s_q=s_q)[1] for a in angles]
    assert max(abs(v) for v in nu2) < 1e-6
    for nu_b in (0.05, 0.02):
        sb = O.rate_from_viscosity(nu_b)
        v = [S.hyperviscosity(a, "mrt", s_xx=sb, s_q=O.quartic_s_q(sb))[1] for a in angles]
        assert max(v) - min(v) < 1e-6 and abs(v[0]) > 1e-4
    v = [S.hyperviscosity(a, "mrt", s_xx=s_xx, s_q=g["non_optimized_s_q_printed"])[1] for a in angles]
    assert max(v) - min(v) > 1e-3


def test_nine_point_stencil_unstable_on_the_diagonal():
    """Section 3-a: the 9-point stencil is linearly unstable in the {1,1} direction, which
    the 3- and 5-point stencils (with s_e = 1) are not."""
    s_xx = O.rate_from_viscosity(0.01)
    ks = np.linspace(0.05, math.pi, 80)

    def worst(stencil, direction):
        d = np.array(direction) / np.linalg.norm(direction)
        return max(np.max(np.abs(np.linalg.eigvals(S.fd_symbol(k * d[0], k * d[1], s_xx=s_xx, stencil=stencil))))
                   for k in ks)

    assert worst(9, (1, 1)) > 1.001
    for stencil in (3, 5):
        for direction in ((1, 0), (2, 1), (1, 1)):
            assert worst(stencil, direction) <= 1.0 + 1e-12


# ------------------------------------- the oracle's linear response equals H(k)^n ----

@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("mode", [(1, 0), (2, 1), (1, 1), (3, 2)])
def test_oracle_linear_response_equals_symbol_power(stencil, mode):
    n, steps = 32, 40
    rng = np.random.default_rng(100 + stencil)
    phi0 = (rng.standard_normal(3) + 1j * rng.standard_normal(3)) * 1e-9
    kx, ky = 2 * math.pi * mode[0] / n, 2 * math.pi * mode[1] / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    wave = np.exp(1j * (kx * x + ky * y))
    fields = [np.real(p * wave) for p in phi0]
    kw = dict(s_xx=1.6, s_e=1.1, stencil=stencil)
    out = O.fd_run(*fields, steps, **kw)
    got = np.array([fourier_coeff(f, *mode) for f in out]) * 2 / n ** 2
    expect = np.linalg.matrix_power(S.fd_symbol(kx, ky, **kw), steps) @ phi0
    assert np.max(np.abs(got - expect)) < 1e-6 * np.max(np.abs(expect))


@pytest.mark.parametrize("mode", [(1, 0), (2, 1), (1, 1)])
def test_mrt_linear_response_equals_symbol_power(mode):
    n, steps = 32, 40
    rng = np.random.default_rng(7)
    phi0 = (rng.standard_normal(3) + 1j * rng.standard_normal(3)) * 1e-9
    kx, ky = 2 * math.pi * mode[0] / n, 2 * math.pi * mode[1] / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    wave = np.exp(1j * (kx * x + ky * y))
    df0 = O.mrt_init(*[np.real(p * wave) for p in phi0])
    kw = dict(s_xx=1.6, s_e=1.1, s_q=1.2, s_eps=1.3)
    df = O.mrt_run(df0, steps, **kw)
    f0 = np.array([fourier_coeff(f, *mode) for f in df0])
    got = np.array([fourier_coeff(f, *mode) for f in df])
    expect = np.linalg.matrix_power(S.mrt_symbol(kx, ky, **kw), steps) @ f0
    assert np.max(np.abs(got - expect)) < 1e-6 * np.max(np.abs(expect))


# ------------------------------------------- shear wave 64 x 64 (section 3-a) ----

def _fit_rate(series, t0, t1):
    t = np.arange(t0, t1 + 1)
    return -np.polyfit(t, np.log(series[t0:t1 + 1]), 1)[0]


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_shear_wave_64_decays_at_nu_k2(scheme):
    """A(t) = <J(t), J(0)> / <J(0), J(0)> decays as exp(-Gamma t) with Gamma = nu k^2 up
    to the hyperviscosity term; the decay rate equals the symbol's shear root."""
    nu = 0.02
    s_xx = O.rate_from_viscosity(nu)
    s_q = O.quartic_s_q(s_xx)
    r, x, y = W.shear_wave_y(64, 64, 0.01, 1)
    k = 2 * math.pi / 64
    norm = np.sum(x * x)
    A = [1.0]
    if scheme == "mrt":
        state = O.mrt_init(r, x, y)
        for _ in range(1000):
            state = O.mrt_run(state, 1, s_xx=s_xx, s_q=s_q)
            A.append(np.sum(O.mrt_moments(state)[1] * x) / norm)
        mass = O.mrt_moments(state)[0].sum()
        g_sym = S.shear_gamma(0.0, k, "mrt", s_xx=s_xx, s_q=s_q).real
        tol = 1e-5
    else:
        st = int(scheme[2])
        state = (r, x, y)
        for _ in range(100):
            state = O.fd_run(*state, 10, s_xx=s_xx, stencil=st)
            A.extend([np.nan] * 9 + [np.sum(state[1] * x) / norm])
        mass = state[0].sum()
        g_sym = S.shear_gamma(0.0, k, s_xx=s_xx, stencil=st).real
        tol = 1e-6
    A = np.array(A)
    t = np.arange(100, 1001, 10)
    gamma = -np.polyfit(t, np.log(A[t]), 1)[0]
    assert abs(gamma / g_sym - 1) < tol
    _, nu2 = S.hyperviscosity(math.pi / 2, "mrt" if scheme == "mrt" else "fd", s_xx=s_xx,
                              **({"s_q": s_q} if scheme == "mrt" else {"stencil": int(scheme[2])}))
    assert abs(gamma / k ** 2 - nu) <= abs(nu2) * k * k * 1.01 + 1e-7
    assert abs(mass) < 1e-13


def test_fd_lbm_and_mrt_agree_to_order_k2():
    """Section 2: FD-LBM and MRT share nu, c_s and the bulk viscosity at order k^2; they
    differ at the next order through the hyperviscosity.  Shear waves of wavelength N = 16,
    32, 64 (nu = 0.02, rate from two times past the initial layer): Gamma_FD / Gamma_MRT - 1
    falls by 4 per doubling of N, and equals (nu2_FD - nu2_MRT) k^2 / nu with the printed
    closed forms nu2 = (2 sigma - 3)(2 sigma - 1)/72 (three points) and sigma (2 sigma - 1)/36
    (five points) (sigma = 1/s_xx - 1/2, wave vector along an axis) and the quartic MRT's own
    shear root."""
    nu = 0.02
    s_xx = O.rate_from_viscosity(nu)
    s_q = O.quartic_s_q(s_xx)
    sig = 1.0 / s_xx - 0.5
    nu2_fd3 = (2 * sig - 3) * (2 * sig - 1) / 72
    _, nu2_mrt = S.hyperviscosity(0.0, "mrt", s_xx=s_xx, s_q=s_q)
    ratio = {}
    for n in (16, 32, 64):
        k = 2 * math.pi / n
        t_end = int(round(0.5 / (nu * k * k)))
        t1 = t_end // 5
        r, jx, jy = W.shear_wave_y(n, n, amp=1e-6, m=1)
        rate = {}
        for scheme in ("fd3", "fd5", "mrt"):
            if scheme == "mrt":
                f = O.mrt_run(O.mrt_init(r, jx, jy), t1, s_xx=s_xx, s_q=s_q)
                a1 = O.mrt_moments(f)
                a2 = O.mrt_moments(O.mrt_run(f, t_end - t1, s_xx=s_xx, s_q=s_q))
            else:
                a1 = O.fd_run(r, jx, jy, t1, s_xx=s_xx, stencil=int(scheme[2]))
                a2 = O.fd_run(*a1, t_end - t1, s_xx=s_xx, stencil=int(scheme[2]))
            rate[scheme] = -math.log(float(np.sum(a2[1] * jx)) / float(np.sum(a1[1] * jx))) / (t_end - t1)
        ratio[n] = {s: rate[s] / rate["mrt"] - 1 for s in ("fd3", "fd5")}
        pred = (nu2_fd3 - nu2_mrt) / nu * k * k
        tol = 0.01 if n == 64 else 0.03 if n == 32 else 0.1
        assert abs(ratio[n]["fd3"] / pred - 1) < tol, (n, ratio[n]["fd3"], pred)
    for a, b in ((16, 32), (32, 64)):
        assert 3.8 < ratio[a]["fd3"] / ratio[b]["fd3"] < 4.2
    # five points: nu2 = sigma (2 sigma - 1)/36 is close to MRT's, so the k^4 terms still weigh
    # at N = 32; at N = 64 the difference is within 15 % of the k^2 prediction and ten times
    # smaller than the three-point one
    nu2_fd5 = sig * (2 * sig - 1) / 36
    pred5 = (nu2_fd5 - nu2_mrt) / nu * (2 * math.pi / 64) ** 2
    assert abs(ratio[64]["fd5"] / pred5 - 1) < 0.15, (ratio[64]["fd5"], pred5)
    assert abs(ratio[64]["fd5"]) < abs(ratio[64]["fd3"]) / 10


# ----------------------------------------- Galilean factor (sections 1-a and 2) ----

@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
@pytest.mark.parametrize("direction", [(1, 0), (0, 1), (1, 1), (1, -1)])
def test_galilean_shear_viscosity(scheme, direction):
    """A shear wave whose wave vector is parallel to a uniform velocity V is damped with
    nu_eff = nu (1 - 3 V^2), for D2Q9 (section 1-a) and for FD-LBM (section 2).  Along an
    axis the factor comes from the cubic terms of theta_XY, along a diagonal from those of
    theta_XX, so the four directions pin every velocity-cubic term of both."""
    nu = 0.05
    s_xx = O.rate_from_viscosity(nu)
    if direction == (1, 0):
        nx, ny, T1, T2 = 128, 4, 200, 1200
    elif direction == (0, 1):
        nx, ny, T1, T2 = 4, 128, 200, 1200
    else:
        nx, ny, T1, T2 = 48, 48, 100, 500
    k = 2 * math.pi * math.hypot(direction[0] / nx, direction[1] / ny)
    t = np.array([-direction[1], direction[0]]) / math.hypot(*direction)
    rates = {}
    for V in (0.0, 0.1, 0.2):
        r, x, y = W.shear_wave(nx, ny, 1e-6, direction[0], direction[1], V=V)
        if scheme == "mrt":
            s_q = O.quartic_s_q(s_xx)
            d1 = O.mrt_run(O.mrt_init(r, x, y), T1, s_xx=s_xx, s_q=s_q)
            d2 = O.mrt_run(d1, T2 - T1, s_xx=s_xx, s_q=s_q)
            m1, m2 = O.mrt_moments(d1), O.mrt_moments(d2)
        else:
            st = int(scheme[2])
            m1 = O.fd_run(r, x, y, T1, s_xx=s_xx, stencil=st)
            m2 = O.fd_run(*m1, T2 - T1, s_xx=s_xx, stencil=st)
        a1 = abs(fourier_coeff(t[0] * m1[1] + t[1] * m1[2], *direction))
        a2 = abs(fourier_coeff(t[0] * m2[1] + t[1] * m2[2], *direction))
        rates[V] = math.log(a1 / a2) / (T2 - T1) / k ** 2
    for V in (0.1, 0.2):
        assert abs(rates[V] / rates[0.0] - (1 - 3 * V * V)) < 1.5e-3, (V, rates)


# ----------------------------------------------------- Poiseuille (section 3-c) ----

@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_poiseuille_profile_and_wall_location(scheme):
    """Channel of 15 fluid rows between walls at y = -1/2 and 14 + 1/2, driven by a uniform
    force; the steady profile is a parabola whose zeros sit at the walls to within a few
    hundredths of a node (halfway bounce-back gives xi_m = 0.5, section 3-c), and which
    converges to the analytic parabola as the channel widens."""
    nu = 1 / math.sqrt(108)
    s_xx = O.rate_from_viscosity(nu)
    errs = []
    for ny in (15, 30):
        r, x, y, F = W.poiseuille_profile(4, ny, nu, 0.05)
        exact = x[:, 0].copy()
        if scheme == "mrt":
            d = O.mrt_run(O.mrt_init(r, x, y), 6000, s_xx=s_xx, s_q=O.quartic_s_q(s_xx), walls=True, fx=F)
            u = O.mrt_moments(d)[1][:, 0] + F / 2
        else:
            out = O.fd_run(r, x, y, 6000, s_xx=s_xx, stencil=int(scheme[2]), walls=True, fx=F)
            u = out[1][:, 0] + F / 2
        yy = np.arange(ny)
        c = np.polyfit(yy, u, 2)
        lo, hi = np.sort(np.roots(c).real)
        assert abs(lo + 0.5) < 0.02 and abs(hi - (ny - 0.5)) < 0.02, (ny, lo, hi)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    assert errs[0] < 1e-2 and errs[1] < errs[0]


# -------------------------------------------------- instability is detectable ----

def test_unstable_stencil_grows_and_stable_ones_decay():
    """The 9-point stencil at nu = 0.01 amplifies noise (its symbol has |z| > 1 on the
    diagonal); the same state decays with the 3-point stencil.  This is the growth that
    the nonfinite / max|J| diagnostics of the GPU path must flag."""
    s_xx = O.rate_from_viscosity(0.01)
    r, x, y = W.random_state(24, 24, seed=9, amp=1e-6)
    bad = O.fd_run(r, x, y, 3000, s_xx=s_xx, stencil=9)
    good = O.fd_run(r, x, y, 3000, s_xx=s_xx, stencil=3)
    j0 = np.max(np.abs(x))
    assert not np.all(np.isfinite(bad[1])) or np.max(np.abs(bad[1])) > 10 * j0
    assert np.max(np.abs(good[1])) < j0


# ------------------------------------------------------------- LW-ACM (section 1-b) ----

def printed_lwacm_matrix(k, v, nu):
    """The amplification matrix printed in section 1-b for the LW-ACM step: wave vector along
    x, mean flow v along it, entries to second order in k, acting on (drho, Jx, Jy)."""
    return np.array([
        [1 - 6j * v * k * nu - k * k * (1 + 3 * v * v) / 6, -6j * nu * k - v * k * k, 0],
        [-1j * k * (1 + 3 * v * v) / 3 + v * (1 - 3 * v * k * k), 1 - 2j * k * v - 3 * nu * k * k, 0],
        [0, 0, 1 - 1j * k * v - nu * k * k],
    ])


def _textbook_bgk(r, x, y, steps):
    """f(x, t+1) = f^eq(x - e_k, t) with the D2Q9 polynomial equilibrium (BGK, tau = 1)."""
    ex, ey = O.velocities()
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    br, bx, by = r.copy(), x.copy(), y.copy()
    for _ in range(steps):
        rho = 1.0 + br
        nr, nx_, ny_ = np.zeros_like(br), np.zeros_like(br), np.zeros_like(br)
        for k in range(9):
            ej = ex[k] * bx + ey[k] * by
            fk = w[k] * (rho + 3 * ej + 4.5 * ej * ej / rho - 1.5 * (bx * bx + by * by) / rho) - w[k]
            fk = np.roll(fk, shift=(ey[k], ex[k]), axis=(0, 1))
            nr += fk
            nx_ += ex[k] * fk
            ny_ += ey[k] * fk
        br, bx, by = nr, nx_, ny_
    return br, bx, by


def test_lwacm_reduces_to_textbook_bgk_when_theta_is_zero():
    """nu = 1/6 makes Theta = 1 - 6 nu = 0: the reconstruction is f* = f^eq, textbook BGK with
    tau = 1, on a nonlinear state."""
    r, x, y = W.random_state(10, 9, seed=18, amp=0.03)
    out = O.lwacm_run(r, x, y, 20, nu=1 / 6)
    for u, v in zip(out, _textbook_bgk(r, x, y, 20)):
        assert np.max(np.abs(u - v)) < 1e-15


def test_lwacm_conserves_mass_and_momentum():
    r, x, y = W.random_state(17, 12, seed=19, amp=0.03)
    out = O.lwacm_run(r, x, y, 25, nu=0.03)
    for u, v in zip(out, (r, x, y)):
        assert abs(np.sum(u) - np.sum(v)) < 1e-13


@pytest.mark.parametrize("nu", [0.005, 0.02, 0.1])
def test_lwacm_symbol_matches_printed_matrix_at_rest(nu):
    """Every entry of the symbol equals the printed matrix up to third order in k: the error
    falls by 8 when k halves, and is far below a wrong second-order coefficient."""
    e1 = np.max(np.abs(S.lwacm_symbol(0.02, 0.0, nu=nu) - printed_lwacm_matrix(0.02, 0.0, nu)))
    e2 = np.max(np.abs(S.lwacm_symbol(0.01, 0.0, nu=nu) - printed_lwacm_matrix(0.01, 0.0, nu)))
    # a wrong second-order coefficient c would leave an error of about c k^2
    assert e1 < 0.02 * 0.02 ** 2 and e1 / e2 > 6, (e1, e2)


@pytest.mark.parametrize("v", [0.02, 0.05, 0.1])
def test_lwacm_symbol_matches_printed_flow_entries(v):
    """In a mean flow the printed J columns and shear entry hold to third order.  The printed
    density column does not: at k = 0 it would make H differ from the identity, which mass
    and momentum conservation forbid (a garbled passage); the symbol keeps H(0) = Id."""
    nu = 0.02
    for k in (0.02, 0.01):
        d = S.lwacm_symbol(k, 0.0, nu=nu, vx=v) - printed_lwacm_matrix(k, v, nu)
        assert np.max(np.abs(d[:, 1:])) < 3 * k ** 3, (k, d)
    assert np.max(np.abs(S.lwacm_symbol(0.0, 0.0, nu=nu, vx=v) - np.eye(3))) < 1e-15


@pytest.mark.parametrize("nu", [0.005, 0.02, 0.05])
def test_lwacm_transport_coefficients(nu):
    """Section 1-b: at rest the sound speed is sqrt(2 nu) and its damping nu/2 + 1/12; the shear
    viscosity is nu, and nu - v^2/2 in a mean flow v along k, which also advects it at v."""
    k = 1e-3
    H = S.lwacm_symbol(k, 0.0, nu=nu)
    g = -np.log(np.linalg.eigvals(H[:2, :2]))
    assert np.allclose(sorted(np.abs(g.imag) / k), [math.sqrt(2 * nu)] * 2, rtol=1e-4)
    assert np.allclose(g.real / k ** 2, nu / 2 + 1 / 12, rtol=1e-4)
    assert abs((-np.log(H[2, 2])).real / k ** 2 - nu) < 1e-4 * nu
    for v in (0.3 * math.sqrt(2 * nu), 0.7 * math.sqrt(2 * nu)):
        g = -np.log(S.lwacm_symbol(k, 0.0, nu=nu, vx=v)[2, 2])
        assert abs(g.real / k ** 2 - (nu - v * v / 2)) < 1e-4 * nu, (v, g)
        assert abs(g.imag / k - v) < 1e-6


@pytest.mark.parametrize("nu", [0.01, 0.05])
def test_lwacm_unstable_above_the_sound_speed(nu):
    """nu(v) = nu - v^2/2 turns negative for v > sqrt(2 nu) = c_s: shear waves then grow, in
    the symbol and in the nonlinear oracle."""
    cs = math.sqrt(2 * nu)
    k = 2 * math.pi / 64
    assert abs(S.lwacm_symbol(k, 0.0, nu=nu, vx=0.8 * cs)[2, 2]) < 1
    assert abs(S.lwacm_symbol(k, 0.0, nu=nu, vx=1.25 * cs)[2, 2]) > 1
    amps = {}
    for f in (0.8, 1.25):
        r, x, y = W.shear_wave(64, 4, 1e-6, 1, 0, V=f * cs)
        _, _, jy = O.lwacm_run(r, x, y, 400, nu=nu)
        amps[f] = abs(fourier_coeff(jy, 1, 0)) / abs(fourier_coeff(y, 1, 0))
    assert amps[0.8] < 1 < amps[1.25], amps


@pytest.mark.parametrize("mode", [(1, 0), (2, 1), (1, 1)])
@pytest.mark.parametrize("V", [(0.0, 0.0), (0.05, 0.02)])
def test_lwacm_linear_response_equals_symbol_power(mode, V):
    """A small plane wave on a uniform flow: after 40 steps of the C oracle its Fourier
    amplitudes are the symbol's 40th power applied to the initial ones."""
    n, steps, nu = 32, 40, 0.03
    rng = np.random.default_rng(31)
    phi0 = (rng.standard_normal(3) + 1j * rng.standard_normal(3)) * 1e-9
    kx, ky = 2 * math.pi * mode[0] / n, 2 * math.pi * mode[1] / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    wave = np.exp(1j * (kx * x + ky * y))
    f = [np.real(p * wave) for p in phi0]
    out = O.lwacm_run(f[0], f[1] + V[0], f[2] + V[1], steps, nu=nu)
    got = np.array([fourier_coeff(u, *mode) for u in out]) * 2 / n ** 2
    expect = np.linalg.matrix_power(S.lwacm_symbol(kx, ky, nu=nu, vx=V[0], vy=V[1]), steps) @ phi0
    assert np.max(np.abs(got - expect)) < 1e-6 * np.max(np.abs(expect))


@pytest.mark.parametrize("V", [0.1, 0.2])
def test_lwacm_galilean_shear_viscosity(V):
    """The nonlinear oracle damps a shear wave in a mean flow V along k with nu - V^2/2 (the
    velocity-square dependence that section 3-a shows for this model in Fig. 1)."""
    nu, nx, ny, T1, T2 = 0.05, 128, 4, 200, 1200
    k = 2 * math.pi / nx
    rates = {}
    for v in (0.0, V):
        r, x, y = W.shear_wave(nx, ny, 1e-6, 1, 0, V=v)
        m1 = O.lwacm_run(r, x, y, T1, nu=nu)
        m2 = O.lwacm_run(*m1, T2 - T1, nu=nu)
        rates[v] = math.log(abs(fourier_coeff(m1[2], 1, 0)) / abs(fourier_coeff(m2[2], 1, 0))) / (T2 - T1) / k ** 2
    assert abs(rates[V] / rates[0.0] - (1 - V * V / (2 * nu))) < 2e-3, rates


# ------------------------------------------- walls at a general distance xi (Fig. 6) ----

@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("xi", [0.2, 0.5, 0.7, 1.0])
def test_ghost_rows_continue_a_linear_shear_through_the_wall(stencil, xi):
    """The ghost rows extrapolate linearly with zero velocity on the wall (section 3-b): for a
    shear jx = a (y + xi), zero on the wall at y = -xi, and uniform density, one step with the
    wall equals one step on a taller domain whose extra rows hold that same linear field."""
    nx, ny, extra, a = 6, 12, 6, 1e-3
    fx = 2e-5
    y = np.arange(ny, dtype=float)
    walled = [np.zeros((ny, nx)), np.repeat((a * (y + xi))[:, None], nx, 1), np.zeros((ny, nx))]
    ye = np.arange(-extra, ny, dtype=float)
    tall = [np.zeros((ny + extra, nx)), np.repeat((a * (ye + xi))[:, None], nx, 1), np.zeros((ny + extra, nx))]
    got = O.fd_run(*walled, 1, s_xx=1.4, s_e=1.1, stencil=stencil, walls=True, xi=xi, fx=fx)
    want = O.fd_run(*tall, 1, s_xx=1.4, s_e=1.1, stencil=stencil, walls=True, xi=0.5, fx=fx)
    for g, w in zip(got, want):
        assert np.max(np.abs(g[:4] - w[extra:extra + 4])) < 1e-17


def _channel_wall_location(scheme, xi, ny=15, steps=4000):
    """Fitted zero of the steady Poiseuille profile beyond the first and last rows."""
    nx, nu, uc = 4, 1 / math.sqrt(108), 0.01
    s_xx = O.rate_from_viscosity(nu)
    L = ny - 1 + 2 * xi
    fx = 8 * nu * uc / L ** 2
    y = np.arange(ny, dtype=float)
    u = fx / (2 * nu) * (y + xi) * (ny - 1 + xi - y)
    r, x, z = np.zeros((ny, nx)), np.repeat(u[:, None], nx, 1) - fx / 2, np.zeros((ny, nx))
    if scheme == "mrt":
        d = O.mrt_run(O.mrt_init(r, x, z), steps, s_xx=s_xx, s_q=O.quartic_s_q(s_xx), walls=True, xi=xi, fx=fx)
        prof = O.mrt_moments(d)[1][:, 0] + fx / 2
    else:
        prof = O.fd_run(r, x, z, steps, s_xx=s_xx, s_e=1.0, stencil=int(scheme[2]), walls=True, xi=xi, fx=fx)[1][:, 0]
        prof = prof + fx / 2
    lo, hi = np.sort(np.roots(np.polyfit(y, prof, 2)).real)
    return -lo, hi - (ny - 1)


@pytest.mark.parametrize("scheme", ["fd3", "fd5", "mrt"])
def test_channel_wall_location_tracks_xi(scheme):
    """Fig. 6: in the channel [1 - xi, 15 + xi] the fitted zero of the velocity follows the
    imposed xi (bounce-back alone would stay at 1/2), for FD-LBM with extrapolated ghost rows
    and for MRT with interpolated bounce-back; both walls give the same location."""
    xis = (0.25, 0.5, 0.75, 1.0)
    got = [_channel_wall_location(scheme, xi) for xi in xis]
    for xi, (lo, hi) in zip(xis, got):
        assert abs(lo - hi) < 1e-9
        assert abs(lo - xi) < 0.06, (xi, lo)
    assert all(b[0] > a[0] + 0.15 for a, b in zip(got, got[1:]))


# ------------------------------------- theta terms against the defect of a BGK step ----

def _theta_error(nx, ny, mx, my, V, a=1e-6):
    """theta is the defect of conservation (section 2): one textbook-BGK step (all rates 1)
    from an equilibrium state leaves non-equilibrium moments m - m^eq(rho', J') = -theta_exact
    to first order in the gradients, theta_exact = d_t m^eq + div(flux) with d_t from the
    Euler equations.  For a density wave of amplitude a on a uniform momentum J = V (every
    derivative of J vanishes) the expansion gives, to first order in a,
        theta_E  = -2 J.grad rho                         + 6 |J|^2 (J.grad rho)
        theta_XX = -2/3 (J_x d_x rho - J_y d_y rho)      + 2 (J_x^2 - J_y^2)(J.grad rho)
        theta_XY = -1/3 (J_x d_y rho + J_y d_x rho)      + 2 J_x J_y (J.grad rho)
    where the first column is what section 2 prints (and the oracle evaluates) and the second
    the |J|^2 terms it omits (rho close to 1).  Returns the defect minus (the oracle's theta
    plus those terms) at the wave's mode, in units of |V| a k, for E, XX, XY."""
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    phase = 2 * np.pi * (mx * xx / nx + my * yy / ny)
    r, x, y = a * np.cos(phase), np.full((ny, nx), V[0]), np.full((ny, nx), V[1])
    f1 = O.mrt_run(O.mrt_init(r, x, y), 1, s_xx=1.0, s_e=1.0, s_q=1.0, s_eps=1.0)
    d = np.tensordot(MF.M, f1 - O.mrt_init(*O.mrt_moments(f1)), axes=(1, 0))
    t = O.fd_theta(r, x, y, 3)
    kx, ky = 2 * math.pi * mx / nx, 2 * math.pi * my / ny
    # amplitude of grad rho under the 3-point differences: i a (sin kx, sin ky)
    jg = V[0] * 1j * a * math.sin(kx) + V[1] * 1j * a * math.sin(ky)
    v2 = V[0] ** 2 + V[1] ** 2
    omitted = (6 * v2 * jg, 2 * (V[0] ** 2 - V[1] ** 2) * jg, 2 * V[0] * V[1] * jg)
    w = np.exp(-1j * phase) * 2 / (nx * ny)
    scale = math.hypot(*V) * a * math.hypot(kx, ky)
    return np.array([(-np.sum(d[3 + q] * w) - np.sum(t[q] * w) - omitted[q]) / scale for q in range(3)])


@pytest.mark.parametrize("V", [(0.03, 0.02), (0.05, -0.03), (0.1, 0.07), (0.0, 0.04)])
@pytest.mark.parametrize("wave", [(256, 4, 1, 0), (4, 256, 0, 1), (128, 128, 1, 1), (128, 128, 1, -1)])
def test_theta_density_gradient_terms_are_the_bgk_defect(V, wave):
    """Pins the density-gradient terms -2 v.grad rho, -2/3 (v_x d_x rho - v_y d_y rho) and
    -1/3 (v_x d_y rho + v_y d_x rho) of theta_E, theta_XX and theta_XY against the defect of
    a textbook-BGK step.  The error at wave vectors k and k/2 is extrapolated to k = 0 (the
    step's second-order terms are O(k)); what is left is O(k^2), below 1e-3 of |V| a k,
    while a wrong coefficient or sign leaves an error of order one."""
    nx, ny, mx, my = wave
    e1 = _theta_error(nx, ny, mx, my, V)
    e2 = _theta_error(2 * nx if nx > 4 else nx, 2 * ny if ny > 4 else ny, mx, my, V)
    assert np.all(np.abs(2 * e2 - e1) < 1e-3), 2 * e2 - e1


# ----------------------------- bulk viscosity in a mean flow (section 2, reading R6) ----
#
# Section 2 states that with its moments the viscosities in a mean flow V are nu (1 - 3V^2)
# (shear, pinned above) and zeta (1 - 3V^2) (bulk), zeta = (1/s_e - 1/2)/3.  The bulk part is
# the coefficient of zeta in the damping of the two sound waves, which only the velocity-cubic
# term of theta_E reaches.  With theta_E = (2 + c|J|^2) div J - 2 J.grad rho that coefficient
# is exactly (1 + c V^2/2)/2 per unit k^2 at every angle between V and k, so the statement
# fixes c = -6 (the printed +6 gives (1 + 3V^2)/2, the opposite sign).

def _acoustic_mean_damping(H, kx, ky, populations=False):
    """Mean Re Gamma of the two acoustic roots (the hydrodynamic roots with more than half of
    their weight in drho and the longitudinal momentum)."""
    z, vec = np.linalg.eig(H)
    k = math.hypot(kx, ky)
    out = []
    for i in np.argsort(-np.abs(z))[:3]:
        m = MF.M[:3] @ vec[:, i] if populations else vec[:, i]
        if (abs(m[0]) + abs(m[1] * kx / k + m[2] * ky / k)) / np.linalg.norm(m) > 0.5:
            out.append(-np.log(z[i]).real)
    assert len(out) == 2, out
    return 0.5 * (out[0] + out[1])


def _bulk_coefficient(damping, ks, zetas=(0.1, 0.2)):
    """d(mean acoustic damping)/d zeta per unit k^2, extrapolated to k = 0 from two wave
    numbers k and k/2 (Richardson: the next terms are O(k^2))."""
    b = []
    for k in ks:
        g = [damping(k, z) / (k * k) for z in zetas]
        b.append((g[1] - g[0]) / (zetas[1] - zetas[0]))
    return (4 * b[1] - b[0]) / 3


def _rate(zeta):
    return 1.0 / (0.5 + 3.0 * zeta)


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("V", [0.05, 0.1, 0.2])
@pytest.mark.parametrize("vang,kang", [(0.0, 0.0), (0.0, math.pi / 4), (math.pi / 2, 0.0),
                                       (math.pi / 4, math.pi / 4), (0.3, 1.1)])
def test_symbol_bulk_viscosity_in_a_mean_flow(stencil, V, vang, kang):
    """The symbol linearised about J = V: the zeta coefficient of the sound damping is
    (1 - 3V^2)/2 at every angle between V and k (section 2), for both stencils; and the
    sound waves are advected at V (phase speeds V.k/|k| +- 1/sqrt 3)."""
    s_xx = O.rate_from_viscosity(0.05)
    vx, vy = V * math.cos(vang), V * math.sin(vang)

    def damping(k, zeta):
        kx, ky = k * math.cos(kang), k * math.sin(kang)
        H = S.fd_symbol(kx, ky, s_xx=s_xx, s_e=_rate(zeta), stencil=stencil, vx=vx, vy=vy)
        return _acoustic_mean_damping(H, kx, ky)

    B = _bulk_coefficient(damping, (0.01, 0.005))
    assert abs(2 * B - (1 - 3 * V * V)) < 1e-6, 2 * B
    # advection of the acoustic pair: mean phase speed V.k/|k|, half-difference c_s
    k = 1e-3
    kx, ky = k * math.cos(kang), k * math.sin(kang)
    z = np.linalg.eigvals(S.fd_symbol(kx, ky, s_xx=s_xx, s_e=1.3, stencil=stencil, vx=vx, vy=vy))
    w = np.sort(-np.angle(z)) / k   # phase speeds of the three roots
    vk = vx * math.cos(kang) + vy * math.sin(kang)
    assert abs(0.5 * (w[0] + w[2]) - vk) < 1e-5 and abs(0.5 * (w[2] - w[0]) - 1 / math.sqrt(3)) < 1e-5


@pytest.mark.parametrize("V", [0.1, 0.2])
def test_d2q9_bulk_viscosity_averages_to_the_stated_factor(V):
    """'As is known for D2Q9' (section 2): the MRT D2Q9 scheme, which has no theta term, damps
    sound in a mean flow with a zeta coefficient that depends on the angle phi between V and
    k, (1 - 3V^2 - 3/2 V^2 cos 2 phi)/2, whose average over phi is the stated (1 - 3V^2)/2."""
    s_xx = O.rate_from_viscosity(0.05)
    coef = []
    for phi in (0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4):

        def damping(k, zeta, phi=phi):
            H = S.mrt_symbol(k, 0.0, s_xx=s_xx, s_e=_rate(zeta), s_q=1.0, vx=V * math.cos(phi), vy=V * math.sin(phi))
            return _acoustic_mean_damping(H, k, 0.0, populations=True)

        coef.append(2 * _bulk_coefficient(damping, (0.01, 0.005)))
        assert abs(coef[-1] - (1 - 3 * V * V - 1.5 * V * V * math.cos(2 * phi))) < 1e-6
    assert abs(np.mean(coef) - (1 - 3 * V * V)) < 1e-6


def _oracle_flow_symbol(step, n, mode, V, s_e, eps=1e-6, **kw):
    """3x3 amplification matrix of one step of the nonlinear oracle about the uniform state
    rho = 1, J = V, by central differences: column j is the response at the wave's mode to
    a plane wave of amplitude eps in field j (the step is translation invariant, so the mode
    maps to itself; the conjugate mode does not reach it)."""
    nx, ny = n if isinstance(n, tuple) else (n, n)
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    phase = 2 * np.pi * (mode[0] * x / nx + mode[1] * y / ny)
    wave = np.cos(phase)
    H = np.zeros((3, 3), dtype=complex)
    for j in range(3):
        resp = []
        for sgn in (1.0, -1.0):
            f = [np.zeros((ny, nx)), np.full((ny, nx), V[0]), np.full((ny, nx), V[1])]
            f[j] = f[j] + sgn * eps * wave
            resp.append(step(*f, s_e=s_e, **kw))
        for i in range(3):
            d = (resp[0][i] - resp[1][i]) / (2 * eps)
            H[i, j] = np.sum(d * np.exp(-1j * phase)) * 2 / (nx * ny)
    return H


def _c_oracle_step(drho, jx, jy, *, s_e, s_xx, stencil):
    return O.fd_run(drho, jx, jy, 1, s_xx=s_xx, s_e=s_e, stencil=stencil)


def _oracle_bulk_error(step, V, direction, stencil=3):
    """2 B - (1 - 3V^2) for the nonlinear oracle `step`, V along `direction`, k along x (on
    N x 4 grids) or along the diagonal (on N x N grids), N = 64 and 128."""
    s_xx = O.rate_from_viscosity(0.05)
    u = np.array(direction, dtype=float) / math.hypot(*direction)
    vel = (V * u[0], V * u[1])

    out = {}
    for kdiag in (False, True):
        def damping(k, zeta, kdiag=kdiag):
            n = int(round(2 * math.pi / (k / math.sqrt(2) if kdiag else k)))
            dims, mode = ((n, n), (1, 1)) if kdiag else ((n, 4), (1, 0))
            H = _oracle_flow_symbol(step, dims, mode, vel, _rate(zeta), s_xx=s_xx, stencil=stencil)
            kx = 2 * math.pi / n
            return _acoustic_mean_damping(H, kx, kx if kdiag else 0.0)

        k1 = 2 * math.pi / 64 * (math.sqrt(2) if kdiag else 1.0)
        out[kdiag] = 2 * _bulk_coefficient(damping, (k1, k1 / 2)) - (1 - 3 * V * V)
    return out


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("mode,V", [((1, 0), (0.1, 0.0)), ((1, 1), (0.07, -0.05)), ((1, 0), (0.15, 0.1))])
def test_oracle_linearised_in_a_mean_flow_equals_the_symbol(stencil, mode, V):
    """The C oracle's own amplification matrix about a uniform flow (central differences of
    one nonlinear step) equals the symbol's, at s_e != 1 where theta_E acts: every velocity
    term of the theta expressions enters the comparison."""
    n = 32
    kx, ky = 2 * math.pi * mode[0] / n, 2 * math.pi * mode[1] / n
    kw = dict(s_xx=1.6, stencil=stencil)
    H = _oracle_flow_symbol(_c_oracle_step, n, mode, V, 1.3, **kw)
    want = S.fd_symbol(kx, ky, s_e=1.3, vx=V[0], vy=V[1], **kw)
    assert np.max(np.abs(H - want)) < 1e-8


@pytest.mark.parametrize("V", [0.1, 0.2])
def test_oracle_bulk_viscosity_in_a_mean_flow(V):
    """The nonlinear C oracle itself, V along x and along the diagonal, sound waves along x
    and along the diagonal: the zeta coefficient of the sound damping, extrapolated to k = 0
    from wavelengths 64 and 128, is (1 - 3V^2)/2 (section 2).  The residue of the
    extrapolation is O(k^4), below 1e-5 for both stencils; the printed sign would leave
    6V^2 (6e-2 at V = 0.1)."""
    for stencil in (3, 5):
        for direction in ((1, 0), (1, 1)):
            err = _oracle_bulk_error(_c_oracle_step, V, direction, stencil)
            assert all(abs(e) < 5e-5 for e in err.values()), (stencil, direction, err)


def test_bulk_pin_detects_a_planted_cubic_coefficient(tmp_path):
    """The bulk pin fails for the printed sign and for other coefficients: a copy of the C
    oracle with the velocity-cubic coefficient of theta_E replaced is compiled here, and its
    zeta coefficient misses (1 - 3V^2)/2 by (c + 6) V^2 / 2."""
    import ctypes
    import subprocess

    src = open(os.path.join(os.path.dirname(O.__file__), "fdlbm_oracle.c")).read()
    term = "*te = (2.0 - 6.0 * (ux * ux + uy * uy))"
    assert src.count(term) == 1
    V = 0.1
    for c in ("+6.0", "-9.0", "-3.0"):
        path = tmp_path / f"planted{c[0] == '+'}{c[1]}.c"
        path.write_text(src.replace(term, f"*te = (2.0 {c[0]} {c[1:]} * (ux * ux + uy * uy))"))
        lib_path = str(path) + ".so"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-o", lib_path,
                        str(path), "-lm"], check=True)
        lib = ctypes.CDLL(lib_path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_fd_step.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 5 + [dp] * 3 + [ctypes.c_int64]

        def step(drho, jx, jy, *, s_e, s_xx, stencil, lib=lib):
            a = [np.ascontiguousarray(f, dtype=np.float64).copy() for f in (drho, jx, jy)]
            ny, nx = a[0].shape
            rc = lib.oracle_fd_step(nx, ny, stencil, 0, 0.5, s_e, s_xx, 0.0, 0.0,
                                    *(f.ctypes.data_as(dp) for f in a), 1)
            assert rc == 0
            return a

        err = _oracle_bulk_error(step, V, (1, 0))
        want = (float(c) + 6.0) * V * V / 2
        for e in err.values():
            assert abs(e - want) < 5e-5 and abs(e) > 100 * 5e-5, (c, err)
