"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and the bench.

This module only draws numbers and lays them out; it holds none of the scheme's
arithmetic (no equilibria, no finite differences, no relaxation).  Both the CPU
oracle and the HIP path receive the arrays built here as plain inputs.

Every field is a float64 array of shape (ny, nx) with x fastest, i.e. element
[j, i] is node (x=i, y=j).  The stored state of a node is the deviation from the
rest state: drho = rho - 1, jx, jy (momentum components).

Workloads (the paper measures only synthetic flows, section 3):
  * plane shear waves (section 3-a), optionally carried by a uniform velocity V;
  * band-limited random Fourier fields ("Stokes modes" / decaying flow);
  * the steady Poiseuille channel profile (section 3-c);
  * the Stokes eigenmodes of a disk with a no-slip wall (section 3-b);
  * a seeded family of independent shear-wave instances of uneven sizes.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "shear_wave",
    "shear_wave_y",
    "fourier_field",
    "stokes_modes_256",
    "decaying_flow",
    "poiseuille_profile",
    "batch_instances",
    "random_state",
    "disk_mode_wavenumber",
    "disk_stokes_mode",
]


def shear_wave(nx, ny, amp, mx, my, V=0.0):
    """Transverse plane wave of integer wave numbers (mx, my) (section 3-a).

    k = 2*pi*(mx/nx, my/ny); the velocity amplitude A(0)=amp is carried by the
    direction perpendicular to k, and an optional uniform velocity V is added
    parallel to k:
        rho = 1,  jx = -amp*ky/|k| cos(k.x) + V kx/|k|,  jy = amp*kx/|k| cos(k.x) + V ky/|k|.
    (The printed initial condition repeats k_x in the phase; the phase is k.x.)
    """
    kx = 2.0 * math.pi * mx / nx
    ky = 2.0 * math.pi * my / ny
    k = math.hypot(kx, ky)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    phase = np.cos(kx * x + ky * y)
    drho = np.zeros((ny, nx))
    jx = -amp * (ky / k) * phase + V * kx / k
    jy = amp * (kx / k) * phase + V * ky / k
    return drho, jx, jy


def shear_wave_y(nx, ny, amp=0.01, m=1):
    """jx(y) = amp*sin(2*pi*m*y/ny), rho = 1, jy = 0 (the 64x64 shear-wave case)."""
    y = np.arange(ny, dtype=np.float64)
    col = amp * np.sin(2.0 * math.pi * m * y / ny)
    jx = np.repeat(col[:, None], nx, axis=1)
    return np.zeros((ny, nx)), jx, np.zeros((ny, nx))


def fourier_field(nx, ny, kmax, rng, row_chunk=2048):
    """Real field made of every Fourier mode 0 < |k| <= kmax (integer wave numbers).

    The coefficients are iid complex Gaussians, i.e. the spectrum of white noise
    with every mode outside the band (and the mean) removed.  The sum is
    evaluated as Re(Ey @ C @ Ex^T) so that an 8192^2 field needs no full FFT.
    The result is not normalised.
    """
    ks = np.arange(-kmax, kmax + 1)
    KY, KX = np.meshgrid(ks, ks, indexing="ij")
    mask = (KX * KX + KY * KY <= kmax * kmax) & ((KX != 0) | (KY != 0))
    c = (rng.standard_normal(KX.shape) + 1j * rng.standard_normal(KX.shape)) * mask
    ex = np.exp(2j * math.pi * np.outer(np.arange(nx), ks) / nx)  # (nx, nk)
    ey = np.exp(2j * math.pi * np.outer(np.arange(ny), ks) / ny)  # (ny, nk)
    a = ey @ c  # (ny, nk)
    ar, ai = np.ascontiguousarray(a.real), np.ascontiguousarray(a.imag)
    exr, exi = ex.real.T.copy(), ex.imag.T.copy()
    out = np.empty((ny, nx))
    for j0 in range(0, ny, row_chunk):
        j1 = min(ny, j0 + row_chunk)
        out[j0:j1] = ar[j0:j1] @ exr - ai[j0:j1] @ exi
    return out


def stokes_modes_256(seed=2, n=256, kmax=8, rms=1e-3):
    """Band-limited random state: each of (drho, jx, jy) holds the modes 0<|k|<=kmax
    and is rescaled to the given RMS."""
    rng = np.random.default_rng(seed)
    fields = []
    for _ in range(3):
        f = fourier_field(n, n, kmax, rng)
        fields.append(f * (rms / np.sqrt(np.mean(f * f))))
    return tuple(fields)


def decaying_flow(n=8192, seed=4, kmax=32, amp=0.02, ny=None):
    """Large decaying flow: per field, random modes 0<|k|<=kmax scaled to max|field|=amp."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    fields = []
    for _ in range(3):
        f = fourier_field(n, ny, kmax, rng)
        fields.append(f * (amp / np.max(np.abs(f))))
    return tuple(fields)


def poiseuille_profile(nx, ny, nu, u_c=0.05):
    """Channel with walls at y=-1/2 and y=ny-1/2 (x periodic), centre-line speed u_c.

    Returns (drho, jx, jy, force_x): the parabola u(y) = F/(2 nu) (y+1/2)(ny-1/2-y),
    with the body force F = 8 nu u_c / ny^2 that sustains it.
    """
    F = 8.0 * nu * u_c / (ny * ny)
    y = np.arange(ny, dtype=np.float64)
    u = F / (2.0 * nu) * (y + 0.5) * (ny - 0.5 - y)
    jx = np.repeat(u[:, None], nx, axis=1)
    return np.zeros((ny, nx)), jx, np.zeros((ny, nx)), F


def batch_instances(count=512, seed=5, nmin=32, nmax=1024, numin=0.005, numax=0.1, mmax=4):
    """Independent shear-wave instances of uneven size and viscosity.

    N ~ U{nmin..nmax}, nu ~ U[numin, numax], m ~ U{1..mmax}; each instance starts
    from jx = 0.01 sin(2 pi m y / N), drho = jy = 0 on an N x N periodic grid.
    """
    rng = np.random.default_rng(seed)
    n = rng.integers(nmin, nmax + 1, size=count)
    nu = rng.uniform(numin, numax, size=count)
    m = rng.integers(1, mmax + 1, size=count)
    return [dict(n=int(n[i]), nu=float(nu[i]), m=int(m[i]), amp=0.01) for i in range(count)]


def random_state(nx, ny, seed, amp=1e-2):
    """Uniform white noise of amplitude amp in each field (small parity cases)."""
    rng = np.random.default_rng(seed)
    return tuple(amp * (2.0 * rng.random((ny, nx)) - 1.0) for _ in range(3))


def disk_mode_wavenumber(m, l, R):
    """k = j_{m+1,l} / R: the l-th Stokes eigenmode of azimuthal order m in a disk of radius
    R with a no-slip wall decays as exp(-nu k^2 t) (section 3-b).  The stream function
    psi = [J_m(k r) - J_m(k R) (r/R)^m] cos(m theta) needs psi(R) = psi'(R) = 0, which
    reduces to J_{m+1}(k R) = 0 (Bessel recurrence); m = 0 gives the singlets (zeros of
    J_1), m >= 1 the doublets (first zero of J_{m+1} for the l-th doublet, l = m)."""
    from scipy.special import jn_zeros

    return float(jn_zeros(m + 1, l)[-1]) / R


def disk_stokes_mode(nx, ny, cx, cy, R, m, k, amp=1e-3, nu=None):
    """Velocity of the Stokes mode psi = [J_m(k r) - J_m(k R) (r/R)^m] cos(m theta) of a
    disk of radius R centred at (cx, cy), scaled to max |J| = amp over the nodes with r < R
    and zero elsewhere: J = (d psi/dy, -d psi/dx).  With nu given, drho carries the pressure
    that keeps the mode incompressible as it decays: the harmonic part B r^m cos(m theta)
    (B = -J_m(kR)/R^m) is the gradient of phi = -B r^m sin(m theta), so drho = 3 nu k^2 phi
    (c_s^2 = 1/3); the Bessel part needs none.  (cx, cy) must not be a node."""
    from scipy.special import jv, jvp

    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    X, Y = x - cx, y - cy
    r = np.hypot(X, Y)
    if np.min(r) == 0.0:
        raise ValueError("the disk centre must not be a node")
    th = np.arctan2(Y, X)
    b = jv(m, k * R) / R ** m
    F = jv(m, k * r) - b * r ** m
    dF = k * jvp(m, k * r) - (m * b * r ** (m - 1) if m > 0 else 0.0)
    c, s = np.cos(m * th), np.sin(m * th)
    dpsi_dx = dF * c * np.cos(th) + m * F / r * s * np.sin(th)
    dpsi_dy = dF * c * np.sin(th) - m * F / r * s * np.cos(th)
    inside = r < R
    scale = amp / np.max(np.hypot(dpsi_dx, dpsi_dy)[inside])
    jx = np.where(inside, scale * dpsi_dy, 0.0)
    jy = np.where(inside, -scale * dpsi_dx, 0.0)
    drho = np.zeros((ny, nx))
    if nu is not None and m > 0:
        drho = np.where(inside, 3.0 * nu * k * k * scale * b * r ** m * s, 0.0)
    return drho, jx, jy


# ------------------------------------------------------------- three dimensions (D3Q19) ----

def random_state3(nx, ny, nz, seed, amp=1e-2):
    """Uniform white noise of amplitude amp in each of (drho, jx, jy, jz), shape (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    return tuple(amp * (2.0 * rng.random((nz, ny, nx)) - 1.0) for _ in range(4))


def decaying_flow3(n, seed=6, kmax=8, amp=0.02, dtype=np.float64):
    """Band-limited random state on an n^3 periodic grid: per field (drho, jx, jy, jz), every
    Fourier mode with 0 < |k| <= kmax (integer wave numbers) with a random complex amplitude,
    scaled to max|field| = amp.  The three-dimensional counterpart of decaying_flow."""
    rng = np.random.default_rng(seed)
    kk = np.fft.fftfreq(n, 1.0 / n)
    kr = np.arange(n // 2 + 1)
    k2 = kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kr[None, None, :] ** 2
    mask = (k2 > 0) & (k2 <= kmax * kmax)
    out = []
    for _ in range(4):
        spec = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
        cnt = int(mask.sum())
        spec[mask] = rng.standard_normal(cnt) + 1j * rng.standard_normal(cnt)
        f = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
        f *= amp / np.max(np.abs(f))
        out.append(np.ascontiguousarray(f.astype(dtype)))
        del spec
    return tuple(out)


def plane_wave3(shape, m, field, amp=1e-6, V=(0.0, 0.0, 0.0)):
    """cos(k.x) of amplitude amp in one field (0 = drho, 1-3 = J components) on the uniform
    state rho = 1, J = V; k = 2 pi (mx/nx, my/ny, mz/nz), shape (nz, ny, nx)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = 2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)
    st = [np.zeros(shape)] + [np.full(shape, float(v)) for v in V]
    st[field] = st[field] + amp * np.cos(ph)
    return tuple(st)
