"""Pins of the D3Q19 FD-LBM oracle against what the mathematics fixes.

The paper's Conclusion says the section-2 analysis was also carried out for D3Q19 and prints
no expression; the oracle applies section 2's construction to D3Q19 (readings D1-D5 in its
header).  Each test below checks it against something other than itself: lattice isotropy,
orthogonality of the moment basis, exact invariants, the reduction to textbook D3Q19 BGK at
unit rates, the independently written linear symbol, the transport coefficients of a
brute-force D3Q19 MRT at order k^2, the Galilean factor nu (1 - 3V^2) and the bulk factor
(1 - 3V^2) that section 2 states for its model, and the defect of conservation that one BGK
step leaves.  No GPU is used.
"""
import math
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import d3q19 as D

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------- textbook D3Q19 (the tests' own) ----

def _textbook_lattice():
    """The 19 velocities with |c|^2 <= 2 and the standard weights, in the oracle's order."""
    cx, cy, cz = (a.astype(float) for a in D.velocities())
    c = np.stack([cx, cy, cz], axis=1)
    c2 = np.sum(c * c, axis=1)
    w = np.choose(c2.astype(int), [1 / 3, 1 / 18, 1 / 36])
    return c, w


def _bgk_feq(c, w, rho, J):
    """Second-order polynomial equilibrium, deviations from the rest populations."""
    cu = np.tensordot(c, J, axes=(1, 0))
    j2 = np.sum(J * J, axis=0)
    return w[:, None, None, None] * (rho - 1 + 3 * cu + 4.5 * cu * cu / rho - 1.5 * j2 / rho)


def _stream(c, f):
    return np.stack([np.roll(f[q], shift=(int(c[q, 2]), int(c[q, 1]), int(c[q, 0])), axis=(0, 1, 2))
                     for q in range(19)])


def _moments(c, f):
    return np.sum(f, axis=0), np.tensordot(c.T, f, axes=(1, 0))


def _fourier(field, m):
    nz, ny, nx = field.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.sum(field * np.exp(-2j * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz))) * 2 / field.size


# ----------------------------------------------------------------- lattice and moments ----

def test_velocity_set_and_weights_are_isotropic_to_fourth_order():
    c, w = _textbook_lattice()
    assert len({tuple(v) for v in c}) == 19
    assert all(tuple(-v) in {tuple(u) for u in c} for v in c)
    assert abs(w.sum() - 1) < 1e-15
    d = np.eye(3)
    assert np.allclose(np.einsum("q,qa,qb->ab", w, c, c), d / 3, atol=1e-15)
    four = np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(four, iso, atol=1e-15)
    assert np.allclose(np.einsum("q,qa,qb,qc->abc", w, c, c, c), 0)


def test_moment_basis_is_orthogonal_with_the_conserved_rows_first():
    """The 19 rows are mutually orthogonal; rho, j_x, j_y, j_z are the rows 1, c_x, c_y, c_z;
    the six second-order rows span the quadratic polynomials orthogonal to 1 (with e = 19|c|^2
    - 30 carrying the trace); the rest are of higher order."""
    c, _ = _textbook_lattice()
    M = D.moment_matrix()
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=1e-12)
    assert np.allclose(M[0], 1) and np.allclose(M[3], c[:, 0]) and np.allclose(M[5], c[:, 1])
    assert np.allclose(M[7], c[:, 2])
    quad = np.array([c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)])  # 6 quadratics
    second = M[[1, 9, 11, 13, 14, 15]]
    # every quadratic is a combination of rho and the second-order rows, and vice versa
    basis = np.vstack([M[0], second])
    coef, res, *_ = np.linalg.lstsq(basis.T, quad.T, rcond=None)
    assert np.allclose(basis.T @ coef, quad.T, atol=1e-12)
    assert np.allclose(M[1], 19 * np.sum(c * c, axis=1) - 30)
    # the other rows are orthogonal to every polynomial of degree <= 2
    others = [r for r in range(19) if r not in (0, 1, 3, 5, 7, 9, 11, 13, 14, 15)]
    lin = np.vstack([np.ones(19), c.T, quad])
    assert np.allclose(M[others] @ lin.T, 0, atol=1e-12)


# ----------------------------------------------------------------- exact invariants ----

def test_uniform_states_are_fixed_points():
    shape = (5, 4, 6)
    st = [np.full(shape, v) for v in (0.01, 0.03, -0.02, 0.015)]
    out = D.fd3d_run(*st, 3, s_nu=1.3, s_e=1.1)
    for a, b in zip(out, st):
        assert np.max(np.abs(a - b)) < 1e-16


def test_mass_and_momentum_are_conserved():
    st = W.random_state3(7, 6, 5, seed=11, amp=0.03)
    out = D.fd3d_run(*st, 5, s_nu=1.7, s_e=1.2)
    for a, b in zip(out, st):
        assert abs(a.sum() - b.sum()) < 1e-14


def test_unit_rates_reduce_to_textbook_bgk():
    """At s_nu = s_e = 1 the defects carry the factor 1 - 1/s = 0, so f* is the equilibrium
    and the step is textbook D3Q19 BGK with tau = 1, f(x, t+1) = f^eq(x - c, t)."""
    c, w = _textbook_lattice()
    st = W.random_state3(6, 5, 7, seed=12, amp=0.03)
    rho, J = 1 + st[0], np.stack(st[1:])
    for _ in range(8):
        f = _stream(c, _bgk_feq(c, w, rho, J))
        dr, J = _moments(c, f)
        rho = 1 + dr
    out = D.fd3d_run(*st, 8, s_nu=1.0, s_e=1.0)
    assert np.max(np.abs(out[0] - (rho - 1))) < 1e-15
    for a in range(3):
        assert np.max(np.abs(out[1 + a] - J[a])) < 1e-15


# ------------------------------------------------ linear response against the symbol ----

@pytest.mark.parametrize("m,shape,V", [
    ((1, 0, 0), (3, 3, 16), (0.0, 0.0, 0.0)),
    ((1, 2, 0), (3, 8, 8), (0.05, -0.03, 0.02)),
    ((1, 1, 1), (8, 8, 8), (0.04, 0.02, -0.05)),
    ((2, -1, 3), (12, 8, 10), (-0.06, 0.0, 0.03)),
])
def test_oracle_linear_response_equals_symbol(m, shape, V):
    """One oracle step of a plane wave of amplitude 1e-6 in each field, on the uniform state
    rho = 1, J = V: its Fourier coefficients equal the symbol's column (the rest is the
    nonlinear O(amplitude) part)."""
    nz, ny, nx = shape
    k = 2 * np.pi * np.array([m[0] / nx, m[1] / ny, m[2] / nz])
    H = D.fd3d_symbol(k, s_nu=1.4, s_e=1.25, V=V)
    amp = 1e-6
    for fld in range(4):
        st = W.plane_wave3(shape, m, fld, amp=amp, V=V)
        out = D.fd3d_run(*st, 1, s_nu=1.4, s_e=1.25)
        got = np.array([_fourier(out[q] - (0 if q == 0 else V[q - 1]), m) for q in range(4)]) / amp
        assert np.max(np.abs(got - H[:, fld])) < 1e-5, (fld, got, H[:, fld])


# ------------------------------------------------------------ transport coefficients ----

DIRS = [(1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 2, 3)]


def _roots(H, k, V):
    """The four hydrodynamic rates Gamma = -log z: two shear roots (advected at k.V), then
    two sound roots."""
    g = -np.log(np.linalg.eigvals(H))
    kv = float(np.dot(k, V))
    order = np.argsort(np.abs(g.imag - kv))
    shear, sound = g[order[:2]], g[order[2:]]
    # a fixed order within each pair, so that roots at k and k/2 are paired
    return shear[np.argsort(shear.real)], sound[np.argsort(sound.imag)]


def _richardson(f, k0):
    """f(k)/k^2 extrapolated to k = 0 from k0 and k0/2 (the next terms are O(k^2))."""
    a, b = f(k0), f(k0 / 2)
    return (4 * b - a) / 3


@pytest.mark.parametrize("s_nu,s_e", [(1.2, 1.4), (1.8, 1.1), (0.9, 1.6)])
@pytest.mark.parametrize("d", DIRS)
def test_symbol_transport_coefficients(s_nu, s_e, d):
    """Shear viscosity nu = (1/s_nu - 1/2)/3 for both shear roots, sound speed 1/sqrt 3,
    sound damping (2/3) nu + zeta/2 with the D3Q19 bulk viscosity zeta = (2/9)(1/s_e - 1/2),
    in every direction (isotropy at order k^2)."""
    n = np.array(d, float) / np.linalg.norm(d)
    nu, zeta = (1 / s_nu - 0.5) / 3, 2 / 9 * (1 / s_e - 0.5)

    def shear(k):
        sh, _ = _roots(D.fd3d_symbol(k * n, s_nu=s_nu, s_e=s_e), k * n, (0, 0, 0))
        return sh.real / k ** 2

    def sound(k):
        _, sd = _roots(D.fd3d_symbol(k * n, s_nu=s_nu, s_e=s_e), k * n, (0, 0, 0))
        return np.array([np.mean(sd.real) / k ** 2, np.max(np.abs(sd.imag)) / k])

    # at k0 = 0.005 what Richardson leaves is O(k0^4), below 1e-8
    assert np.all(np.abs(_richardson(shear, 0.005) - nu) < 1e-8)
    damp, cs = _richardson(sound, 0.005)
    assert abs(cs - 1 / math.sqrt(3)) < 1e-8
    assert abs(damp - (2 / 3 * nu + zeta / 2)) < 1e-8


def _mrt_symbol(k, s_nu, s_e, V):
    """Brute-force D3Q19 MRT (19 populations; rates s_e on e, s_nu on the five traceless
    second-order rows, 1 on every other non-conserved row, the second-order polynomial
    equilibrium), linearised about (1, V): f -> exp(-i k.c) M^{-1} (M - S (M - M_eq))."""
    c, w = _textbook_lattice()
    M = D.moment_matrix()
    Minv = np.linalg.inv(M)
    V = np.asarray(V, float)
    cu = c @ V
    jac = np.zeros((19, 4))
    jac[:, 0] = w * (1 - 4.5 * cu * cu + 1.5 * V @ V)
    for a in range(3):
        jac[:, 1 + a] = w * (3 * c[:, a] + 9 * cu * c[:, a] - 3 * V[a])
    cons = np.vstack([np.ones(19), c.T])  # rho, J of the populations
    S = np.ones(19)
    S[[0, 3, 5, 7]] = 0
    S[1] = s_e
    S[[9, 11, 13, 14, 15]] = s_nu
    coll = Minv @ (M - np.diag(S) @ (M - M @ jac @ cons))
    return np.exp(-1j * (c @ k))[:, None] * coll


@pytest.mark.parametrize("s_nu,s_e", [(1.2, 1.4), (1.7, 1.05)])
@pytest.mark.parametrize("d", DIRS)
def test_hydrodynamic_roots_equal_brute_force_mrt_at_order_k2(s_nu, s_e, d):
    """Section 2's construction reproduces the moments of the LBM it approximates to second
    order (eq. order2): the four hydrodynamic roots of FD-LBM and of a brute-force D3Q19 MRT
    with the same second-order rates agree at order k^2 (their k^3 and k^4 terms differ)."""
    n = np.array(d, float) / np.linalg.norm(d)

    def roots(sym):
        def f(k):
            g = -np.log(np.linalg.eigvals(sym(k)))
            g = g[np.argsort(np.abs(g))][:4]
            return np.sort_complex(g / k ** 2)
        return f

    fd = _richardson(roots(lambda k: D.fd3d_symbol(k * n, s_nu=s_nu, s_e=s_e)), 0.01)
    mrt = _richardson(roots(lambda k: _mrt_symbol(k * n, s_nu, s_e, (0, 0, 0))), 0.01)
    assert np.max(np.abs(fd.real - mrt.real)) < 1e-6


@pytest.mark.parametrize("d", DIRS)
@pytest.mark.parametrize("v", [0.05, 0.1, 0.2])
def test_galilean_shear_viscosity(d, v):
    """Section 2: in a mean flow V the shear viscosity of the model is nu (1 - 3V^2), here
    for both transverse waves with k parallel to V, in every direction."""
    n = np.array(d, float) / np.linalg.norm(d)
    s_nu = 1.3
    nu = (1 / s_nu - 0.5) / 3

    def shear(k):
        sh, _ = _roots(D.fd3d_symbol(k * n, s_nu=s_nu, s_e=1.2, V=v * n), k * n, v * n)
        return sh.real / k ** 2

    assert np.all(np.abs(_richardson(shear, 0.004) / (nu * (1 - 3 * v * v)) - 1) < 1e-4)


def _bulk_coefficient(H_of, k0, zetas=(1.3, 1.6)):
    """d(mean damping of the two sound roots)/d zeta per unit k^2, extrapolated to k = 0."""
    def f(k):
        g = []
        for s_e in zetas:
            H, kv, V = H_of(k, s_e)
            _, sd = _roots(H, kv, V)
            g.append(np.mean(sd.real) / k ** 2)
        z = [2 / 9 * (1 / s - 0.5) for s in zetas]
        return (g[1] - g[0]) / (z[1] - z[0])
    return _richardson(f, k0)


@pytest.mark.parametrize("d", DIRS)
@pytest.mark.parametrize("v", [0.1, 0.2])
def test_symbol_bulk_viscosity_in_a_mean_flow(d, v):
    """Section 2 states the bulk viscosity in a mean flow as zeta (1 - 3V^2): the coefficient
    of zeta in the sound damping is (1 - 3V^2)/2 for k parallel to V, in every direction.
    Only the velocity-cubic term of the energy defect reaches it (reading D4)."""
    n = np.array(d, float) / np.linalg.norm(d)
    b = _bulk_coefficient(lambda k, s_e: (D.fd3d_symbol(k * n, s_nu=1.25, s_e=s_e, V=v * n), k * n, v * n), 0.004)
    assert abs(b / ((1 - 3 * v * v) / 2) - 1) < 1e-4


def _oracle_H(shape, m, s_nu, s_e, V, lib_run=None):
    """The oracle's own amplification matrix at the lattice wave vector m, from one step of
    four plane waves of amplitude 1e-7."""
    run = lib_run or (lambda st: D.fd3d_run(*st, 1, s_nu=s_nu, s_e=s_e))
    H = np.zeros((4, 4), complex)
    for fld in range(4):
        st = W.plane_wave3(shape, m, fld, amp=1e-7, V=V)
        out = run(st)
        H[:, fld] = [_fourier(out[q] - (0 if q == 0 else V[q - 1]), m) / 1e-7 for q in range(4)]
    return H


def _oracle_bulk(v, run_for=None):
    """Bulk coefficient of the oracle itself (not the symbol) for k and V along x."""
    def H_of(k, s_e):
        nx = int(round(2 * np.pi / k))
        run = None if run_for is None else run_for(s_e)
        H = _oracle_H((3, 3, nx), (1, 0, 0), 1.25, s_e, (v, 0.0, 0.0), run)
        return H, np.array([k, 0, 0]), np.array([v, 0, 0])
    return _bulk_coefficient(H_of, 2 * np.pi / 64)


def test_oracle_bulk_viscosity_in_a_mean_flow():
    v = 0.15
    assert abs(_oracle_bulk(v) / ((1 - 3 * v * v) / 2) - 1) < 2e-3


def test_bulk_pin_detects_a_planted_cubic_coefficient(tmp_path):
    """The same measurement on a copy of the oracle whose energy defect carries -3 |J|^2 div J
    (the coefficient of the exact defect along an axis) instead of -2 misses the stated factor
    by more than the tolerance."""
    src = open(os.path.join(HERE, "..", "oracle", "fd3d_oracle.c")).read()
    planted, n = re.subn(r"- 2\.0 \* j2 \* div", "- 3.0 * j2 * div", src)
    assert n == 1
    cfile = tmp_path / "planted.c"
    cfile.write_text(planted)
    so = tmp_path / "libplanted.so"
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
                    "-o", str(so), str(cfile), "-lm"], check=True)
    import ctypes
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_fd3d_step.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [dp] * 4 + [ctypes.c_int64]

    def run_for(s_e):
        def run(st):
            a = [np.ascontiguousarray(x, dtype=np.float64).copy() for x in st]
            nz, ny, nx = a[0].shape
            assert lib.oracle_fd3d_step(nx, ny, nz, s_e, 1.25, *(x.ctypes.data_as(dp) for x in a), 1) == 0
            return a
        return run

    v = 0.15
    assert abs(_oracle_bulk(v, run_for) / ((1 - 3 * v * v) / 2) - 1) > 1e-2


# ------------------------------------------------ density-gradient terms of theta ----

def _theta_error(shape, m, V, a=1e-6):
    """One textbook-BGK step from the equilibrium of a density wave on a uniform momentum
    J = V leaves non-equilibrium second-order moments equal to minus the exact defect, whose
    expansion to first order in a is, per stress component,
        theta_ab = -1/3 (V_a d_b rho + V_b d_a rho) + 2 V_a V_b (V.grad rho)
    (every derivative of J vanishes).  The oracle evaluates the first part (reading D4, rho
    close to 1); the second is added here.  Returns the error of the six moments at the
    wave's mode in units of |V| a k."""
    c, w = _textbook_lattice()
    M = D.moment_matrix()
    st = W.plane_wave3(shape, m, 0, amp=a, V=V)
    rho, J = 1 + st[0], np.stack(st[1:])
    f1 = _stream(c, _bgk_feq(c, w, rho, J))
    dr1, J1 = _moments(c, f1)
    neq = np.tensordot(M, f1 - _bgk_feq(c, w, 1 + dr1, J1), axes=(1, 0))
    th = D.fd3d_theta(*st)
    nz, ny, nx = shape
    k = 2 * np.pi * np.array([m[0] / nx, m[1] / ny, m[2] / nz])
    g = 1j * a * np.sin(k)  # 3-point gradient of the wave, at its mode
    V = np.asarray(V, float)
    vg = V @ g
    omitted_ab = 2 * np.outer(V, V) * vg
    tr = np.trace(omitted_ab)
    omitted = [19 * tr, 2 * omitted_ab[0, 0] - omitted_ab[1, 1] - omitted_ab[2, 2],
               omitted_ab[1, 1] - omitted_ab[2, 2], omitted_ab[0, 1], omitted_ab[1, 2], omitted_ab[0, 2]]
    rows = [1, 9, 11, 13, 14, 15]
    scale = np.linalg.norm(V) * a * np.linalg.norm(k)
    return np.array([(-_fourier(neq[r], m) - _fourier(th[q], m) - omitted[q]) / scale
                     for q, r in enumerate(rows)])


@pytest.mark.parametrize("V", [(0.03, 0.02, -0.01), (0.05, -0.03, 0.04), (0.0, 0.04, 0.0), (0.08, 0.05, 0.06)])
@pytest.mark.parametrize("wave", [((3, 3, 64), (1, 0, 0)), ((3, 64, 3), (0, 1, 0)), ((64, 3, 3), (0, 0, 1)),
                                  ((3, 64, 64), (1, 1, 0)), ((64, 3, 64), (1, 0, -1))])
def test_theta_density_gradient_terms_are_the_bgk_defect(V, wave):
    """Pins -1/3 (J_a d_b rho + J_b d_a rho) in the five traceless defects and -2/3 J.grad rho
    in the energy defect against the defect of a textbook-BGK step, extrapolated to k = 0 from
    k and k/2 (the step's own second-order terms are O(k))."""
    shape, m = wave
    shape2 = tuple(2 * s if s > 3 else s for s in shape)
    e1 = _theta_error(shape, m, V)
    e2 = _theta_error(shape2, m, V)
    # per unit of the stress: e = 19 tr Pi - 30 rho and 3p_xx = 3 Pi_xx - tr Pi carry factors
    # 19 and 3; a wrong coefficient or sign leaves an error of order one per unit
    unit = np.array([19, 3, 1, 1, 1, 1])
    assert np.all(np.abs(2 * e2 - e1) / unit < 1e-3), 2 * e2 - e1


# ------------------------------------------------------------------ nonlinear runs ----

def test_shear_wave_decays_at_the_symbol_rate():
    """A transverse wave of amplitude 1e-4 on a 3 x 3 x 32 grid decays over 300 steps at the
    rate of the symbol's shear root (nonlinear effects are O(amplitude^2) for it)."""
    shape, m, s_nu = (3, 3, 32), (1, 0, 0), 1.6
    st = W.plane_wave3(shape, m, 2, amp=1e-4)
    out = D.fd3d_run(*st, 300, s_nu=s_nu, s_e=1.3)
    k = np.array([2 * np.pi / 32, 0, 0])
    sh, _ = _roots(D.fd3d_symbol(k, s_nu=s_nu, s_e=1.3), k, (0, 0, 0))
    want = 1e-4 * np.exp(-300 * sh[0].real)
    got = abs(_fourier(out[2], m))
    assert abs(got / want - 1) < 1e-6
