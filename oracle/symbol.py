"""Linear amplification matrices of the FD-LBM and MRT D2Q9 schemes (von Neumann analysis).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 1-b: a plane wave of small amplitude, Phi = (drho, J_x, J_y) * p^i q^j with
p = exp(i k_x), q = exp(i k_y), is multiplied by the amplification matrix H after one
step (Phi^{n+1} = H Phi^n); the roots z of det(H - z Id) = 0 give Gamma = -log z.
Section 2 interprets the shear root as Gamma = nu_0 k^2 + nu_2 k^4 ("hyperviscosity" nu_2),
and solves the full cubic numerically up to k = pi for linear stability.

Here H is assembled numerically about a uniform state rho = 1, J = (vx, vy) (the rest state
by default):
  FD-LBM:  H = P(k) diag(exp(-i k.e_k)) M^{-1} L(k), where L(k) maps Phi to the
           linearised post-collision moments (the equilibria and theta terms linearised
           about the uniform state, the finite differences become their Fourier symbols)
           and P(k) takes the conserved moments of the propagated populations;
  MRT:     H = diag(exp(-i k.e_k)) M^{-1} (I - S + S Q) M on the 9 populations, with Q
           the linearised equilibrium map and S the relaxation rates.
About a uniform flow the velocity-cubic terms of theta enter H; the bulk viscosity of the
acoustic pair then carries the factor (1 - 3 V^2) that section 2 states (tests pin this).
"""
from __future__ import annotations

import math

import numpy as np

from .matrix_form import E, M, MINV, STENCILS


def derivative_symbols(kx, ky, stencil):
    """Fourier symbols (Dx, Dy) of the section-2 finite differences: sum_o w_o exp(i k.o)."""
    dx = sum(w * np.exp(1j * (kx * ox + ky * oy)) for ox, oy, w in STENCILS[stencil])
    dy = sum(w * np.exp(1j * (ky * ox + kx * oy)) for ox, oy, w in STENCILS[stencil])
    return dx, dy


def _propagation(kx, ky):
    return np.diag(np.exp(-1j * (kx * E[:, 0] + ky * E[:, 1])))


def fd_symbol(kx, ky, *, s_xx, s_e=1.0, stencil=3, vx=0.0, vy=0.0):
    """3x3 amplification matrix of the FD-LBM step acting on (drho, Jx, Jy), linearised about
    rho = 1, J = (vx, vy).

    Section 2's moments, with v read as J (reading R3) and the sign of the velocity-cubic
    term of theta_E as section 2's bulk viscosity fixes it (reading R6):
      theta_E  = (2 - 6|J|^2) div J - 2 J.grad rho
      theta_XX = 2/3 (D_x J_x - D_y J_y) - 2/3 (J_x D_x rho - J_y D_y rho)
                 - 2 [J_x (D_x J_x^2 + D_y J_x J_y) - J_y (D_x J_x J_y + D_y J_y^2)]
      theta_XY = 1/3 (D_x J_y + D_y J_x) - 1/3 (J_x D_y rho + J_y D_x rho)
                 - J_x (D_x J_x J_y + D_y J_y^2) - J_y (D_x J_x^2 + D_y J_x J_y)
    Every derivative is of a perturbation (the base state is uniform), so each term is
    linearised by freezing its other factors at the base state."""
    Dx, Dy = derivative_symbols(kx, ky, stencil)
    ce, cxx = 1 - 1 / s_e, 1 - 1 / s_xx
    # perturbations of the stored fields and of the product fields, as rows over Phi
    dr, djx, djy = np.eye(3)
    dP, dQ, dR = 2 * vx * djx, 2 * vy * djy, vy * djx + vx * djy   # Jx^2, Jy^2, Jx Jy
    v2 = vx * vx + vy * vy
    th_e = (2 - 6 * v2) * (Dx * djx + Dy * djy) - 2 * (vx * Dx + vy * Dy) * dr
    th_xx = (2 / 3 * (Dx * djx - Dy * djy) - 2 / 3 * (vx * Dx - vy * Dy) * dr
             - 2 * (vx * (Dx * dP + Dy * dR) - vy * (Dx * dR + Dy * dQ)))
    th_xy = (1 / 3 * (Dx * djy + Dy * djx) - 1 / 3 * (vx * Dy + vy * Dx) * dr
             - vx * (Dx * dR + Dy * dQ) - vy * (Dx * dP + Dy * dR))
    # equilibria (section 1-a table) linearised about the base state, plus the theta parts
    L = _equilibrium_jacobian(vx, vy).astype(complex)
    L[3] += ce * th_e
    L[4] += cxx * th_xx
    L[5] += cxx * th_xy
    P = M[:3]
    return P @ _propagation(kx, ky) @ MINV @ L


def mrt_symbol(kx, ky, *, s_xx, s_e=1.0, s_q, s_eps=1.0, vx=0.0, vy=0.0):
    """9x9 amplification matrix of the MRT step acting on the populations, linearised about
    the equilibrium populations of rho = 1, J = (vx, vy)."""
    S = np.diag([0, 0, 0, s_e, s_xx, s_xx, s_q, s_q, s_eps]).astype(float)
    Q = np.zeros((9, 9))
    Q[:, :3] = _equilibrium_jacobian(vx, vy)   # m^eq depends on the conserved moments only
    C = MINV @ (np.eye(9) - S + S @ Q) @ M
    return _propagation(kx, ky) @ C


def _equilibrium_jacobian(vx, vy):
    """d m^eq / d(rho, Jx, Jy) of the section 1-a table at rho = 1, J = (vx, vy)."""
    v2 = vx * vx + vy * vy
    return np.array([
        [1, 0, 0],
        [0, 1, 0],
        [0, 0, 1],
        [-2 - 3 * v2, 6 * vx, 6 * vy],          # E = -2 rho + 3 |J|^2 / rho
        [-(vx * vx - vy * vy), 2 * vx, -2 * vy],  # XX = (Jx^2 - Jy^2) / rho
        [-vx * vy, vy, vx],                      # XY = Jx Jy / rho
        [0, -1, 0],                              # qx = -Jx
        [0, 0, -1],                              # qy = -Jy
        [1 + 3 * v2, -6 * vx, -6 * vy],          # eps = rho - 3 |J|^2 / rho
    ], dtype=float)


def lwacm_symbol(kx, ky, *, nu, vx=0.0, vy=0.0):
    """3x3 amplification matrix of the LW-ACM step (section 1-b) on (drho, Jx, Jy) about the
    uniform state rho = 1, J = (vx, vy).

    f^{n+1}_k(x) = f^eq_k(x - e_k) + Theta (f^eo_k(x) - f^eo_k(x - e_k)), Theta = 1 - 6 nu, so
    a plane wave gives  f^{n+1} = [P (A_eq - Theta A_eo) + Theta A_eo] Phi  with A_eq, A_eo the
    Jacobians of f^eq and f^eo and P = diag(exp(-i k.e_k)).  f^eo keeps the part of m^eq odd
    in J: its rows J and q, which are linear and do not depend on rho."""
    theta = 1.0 - 6.0 * nu
    A_eq = MINV @ _equilibrium_jacobian(vx, vy)
    m_eo = np.zeros((9, 3))
    m_eo[1, 1] = m_eo[2, 2] = 1
    m_eo[6, 1] = m_eo[7, 2] = -1
    A_eo = MINV @ m_eo
    return M[:3] @ (_propagation(kx, ky) @ (A_eq - theta * A_eo) + theta * A_eo)


def _moments3(scheme, v):
    return v if scheme == "fd" else M[:3] @ v


def shear_gamma(kx, ky, scheme="fd", **params):
    """Gamma = -log z of the transverse (shear) root at wave vector (kx, ky)."""
    H = fd_symbol(kx, ky, **params) if scheme == "fd" else mrt_symbol(kx, ky, **params)
    z, V = np.linalg.eig(H)
    k = math.hypot(kx, ky)
    tx, ty = -ky / k, kx / k
    best, score = None, -1.0
    for i in _hydrodynamic_roots(z):
        m = _moments3(scheme, V[:, i])
        norm = np.linalg.norm(m)
        if norm < 1e-12:
            continue
        s = abs(m[1] * tx + m[2] * ty) / norm
        if s > score:
            best, score = i, s
    return -np.log(z[best])


def _hydrodynamic_roots(z):
    """Indices of the three roots of largest modulus (the slow, hydrodynamic modes; the
    other MRT roots decay within a few steps)."""
    return list(np.argsort(-np.abs(z))[:3])


def sound_gammas(kx, ky, scheme="fd", **params):
    """Gamma of the two acoustic roots (the hydrodynamic roots other than the shear one)."""
    H = fd_symbol(kx, ky, **params) if scheme == "fd" else mrt_symbol(kx, ky, **params)
    z, V = np.linalg.eig(H)
    k = math.hypot(kx, ky)
    nx_, ny_ = kx / k, ky / k
    out = []
    for i in _hydrodynamic_roots(z):
        m = _moments3(scheme, V[:, i])
        norm = np.linalg.norm(m)
        if norm < 1e-12:
            continue
        longit = abs(m[0]) + abs(m[1] * nx_ + m[2] * ny_)
        if longit / norm > 0.5:
            out.append(-np.log(z[i]))
    return sorted(out, key=lambda g: g.imag)


def nu_of_k(k, angle, scheme="fd", **params):
    """k-dependent shear viscosity Re(Gamma)/k^2 along direction `angle` (radians)."""
    g = shear_gamma(k * math.cos(angle), k * math.sin(angle), scheme, **params)
    return g.real / (k * k)


def hyperviscosity(angle, scheme="fd", ks=(0.02, 0.04, 0.06, 0.08, 0.1, 0.12), **params):
    """(nu_0, nu_2) from a least-squares fit nu(k) = nu_0 + nu_2 k^2 + nu_4 k^4 + nu_6 k^6."""
    ks = np.asarray(ks, dtype=float)
    nus = np.array([nu_of_k(k, angle, scheme, **params) for k in ks])
    A = np.stack([np.ones_like(ks), ks ** 2, ks ** 4, ks ** 6], axis=1)
    coef, *_ = np.linalg.lstsq(A, nus, rcond=None)
    return coef[0], coef[1]


def max_amplification(scheme="fd", n=64, **params):
    """max |z| over a grid of wave vectors in [-pi, pi]^2 (linear stability map)."""
    ks = np.linspace(-math.pi, math.pi, n)
    worst = 0.0
    for kx in ks:
        for ky in ks:
            if kx == 0 and ky == 0:
                continue
            H = fd_symbol(kx, ky, **params) if scheme == "fd" else mrt_symbol(kx, ky, **params)
            worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(H)))))
    return worst
