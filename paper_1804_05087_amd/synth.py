"""Seeded synthetic plane-Couette velocity fields.

The paper's experiments start from known exact coherent states (EQ1/NCBW in
plane Couette flow, Sec. 3.3) that are not available here. These generators
produce seeded stand-ins in the same box and representation instead:

* ``perturbation_field``: laminar Couette flow U_lam = y e_x (Sec. 3.1) plus a
  random perturbation u' = curl((1-y^2)^2 phi) with a Gaussian spectral
  envelope exp(-(m_x^2+m_z^2+n^2)/8) on the vector potential phi. The curl of
  such a potential is exactly divergence free and vanishes, with its normal
  derivative, at the walls y = +-1.
* ``streak_roll_field``: streamwise-independent rolls and streaks plus a small
  random perturbation, for the large-box workload.

Every array is in the canonical spectral layout shared by the library and
its tests: complex128 ``[3][Nx][Nz/2+1][Ny]`` holding Chebyshev coefficients in
y, Fourier modes m_x in FFT order (index i -> i for i < Nx/2, i - Nx above)
and m_z = 0..Nz/2. Nyquist entries (i = Nx/2, m_z = Nz/2) are zero, the m_z = 0
plane is Hermitian (entry at -m_x is the conjugate of the one at +m_x) and the
(0,0) mode is real.

This module only synthesises inputs. It uses numpy's Chebyshev-series
library (``numpy.polynomial.chebyshev``) for its few polynomial products,
derivatives and integrals, and shares no arithmetic with either the
library's kernels or the CPU reference.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import chebyshev as C


def _mode_numbers(nx: int, nz: int):
    """Integer m_x (FFT order) and m_z (non-negative) of the canonical layout."""
    mx = np.array([i if i < nx // 2 else i - nx for i in range(nx)], dtype=np.int64)
    mz = np.arange(nz // 2 + 1, dtype=np.int64)
    return mx, mz


def _valid_mask(nx: int, nz: int) -> np.ndarray:
    """True where a Fourier mode is kept (Nyquist rows/columns excluded)."""
    m = np.ones((nx, nz // 2 + 1), dtype=bool)
    m[nx // 2, :] = False
    m[:, nz // 2] = False
    return m


def hermitian_project(a: np.ndarray) -> np.ndarray:
    """Make the m_z = 0 plane Hermitian, the (0,0) mode real and Nyquist zero.

    ``a`` has shape [..., Nx, Nz/2+1, Ny]. The entry at +m_x (m_x > 0) is kept
    and its conjugate copied to -m_x.
    """
    a = np.array(a, dtype=np.complex128, copy=True)
    nx = a.shape[-3]
    nzh = a.shape[-2]
    a[..., nx // 2, :, :] = 0.0
    a[..., :, nzh - 1, :] = 0.0
    for i in range(1, nx // 2):
        a[..., nx - i, 0, :] = np.conj(a[..., i, 0, :])
    a[..., 0, 0, :] = a[..., 0, 0, :].real
    return a


def _cheb_integral(p: np.ndarray) -> float:
    """Integral over [-1, 1] of the real Chebyshev series p."""
    q = C.chebint(p)
    return float(C.chebval(1.0, q) - C.chebval(-1.0, q))


def mean_square(u: np.ndarray) -> float:
    """(1/V) * integral of |u|^2 over the box, for a canonical field u.

    By Parseval in x and z this is (1/2) * sum over all Fourier modes of the
    integral over y of |u_m(y)|^2; stored m_z > 0 modes stand for the pair
    (+-m_z) and count twice.
    """
    nzh = u.shape[-2]
    total = 0.0
    for c in range(u.shape[0]):
        for i in range(u.shape[1]):
            for j in range(nzh):
                a = u[c, i, j, :]
                if not np.any(a):
                    continue
                w = 1.0 if j == 0 else 2.0
                sq = C.chebadd(C.chebmul(a.real, a.real), C.chebmul(a.imag, a.imag))
                total += w * _cheb_integral(sq)
    return 0.5 * total


def laminar_field(nx: int, ny: int, nz: int, wall_upper: float = 1.0,
                  wall_lower: float = -1.0) -> np.ndarray:
    """Couette base flow: u = a + b*y with u(1) = wall_upper, u(-1) = wall_lower."""
    u = np.zeros((3, nx, nz // 2 + 1, ny), dtype=np.complex128)
    u[0, 0, 0, 0] = 0.5 * (wall_upper + wall_lower)
    u[0, 0, 0, 1] = 0.5 * (wall_upper - wall_lower)
    return u


def perturbation(nx: int, ny: int, nz: int, lx: float, lz: float, seed: int,
                 energy: float = 1e-2) -> np.ndarray:
    """Divergence-free, no-slip random perturbation with E = (1/2V)int|u'|^2."""
    if ny < 6:
        raise ValueError("perturbation needs Ny >= 6 (vector potential degree Ny-5)")
    alpha = 2.0 * math.pi / lx
    gamma = 2.0 * math.pi / lz
    N = ny - 1
    mx, mz = _mode_numbers(nx, nz)
    nzh = nz // 2 + 1
    rng = np.random.default_rng(seed)
    nphi = N - 3  # phi has degree <= N-4
    n = np.arange(nphi)
    env = np.exp(-(mx[:, None, None] ** 2 + mz[None, :, None] ** 2 + n[None, None, :] ** 2) / 8.0)
    shape = (3, nx, nzh, nphi)
    phi = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * env[None]
    phi = hermitian_project(phi)
    q = np.array([3.0 / 8.0, 0.0, -0.5, 0.0, 1.0 / 8.0])  # (1-y^2)^2
    psi = np.zeros((3, nx, nzh, ny), dtype=np.complex128)
    dpsi = np.zeros_like(psi)
    for c in range(3):
        for i in range(nx):
            for j in range(nzh):
                f = phi[c, i, j]
                re = C.chebmul(q, f.real)
                im = C.chebmul(q, f.imag)
                p = np.zeros(ny, dtype=np.complex128)
                p[: len(re)] += re
                p[: len(im)] += 1j * im
                psi[c, i, j] = p
                d = C.chebder(p.real) + 1j * C.chebder(p.imag)
                dpsi[c, i, j, : len(d)] = d
    ikx = 1j * alpha * mx[:, None, None]
    ikz = 1j * gamma * mz[None, :, None]
    u = np.empty_like(psi)
    u[0] = dpsi[2] - ikz * psi[1]
    u[1] = ikz * psi[0] - ikx * psi[2]
    u[2] = ikx * psi[1] - dpsi[0]
    u = hermitian_project(u)
    e = 0.5 * mean_square(u)
    if e > 0:
        u *= math.sqrt(energy / e)
    return u


def perturbation_field(nx: int, ny: int, nz: int, lx: float, lz: float, seed: int,
                       energy: float = 1e-2, wall_upper: float = 1.0,
                       wall_lower: float = -1.0) -> np.ndarray:
    """Laminar Couette flow plus the seeded perturbation family."""
    return laminar_field(nx, ny, nz, wall_upper, wall_lower) + perturbation(
        nx, ny, nz, lx, lz, seed, energy)


def streak_roll_field(nx: int, ny: int, nz: int, lx: float, lz: float, seed: int = 0,
                      roll_amp: float = 0.05, streak_amp: float = 0.3,
                      noise_rms: float = 1e-3) -> np.ndarray:
    """Laminar flow + streamwise rolls and streaks in the first spanwise mode + noise.

    Rolls: psi = (1-y^2)^2 sin(gamma z), v = d(psi)/dz, w = -d(psi)/dy, with
    max|v| = roll_amp. Streaks: u = -(1-y^2) cos(gamma z), max|u| = streak_amp.
    Noise: the perturbation family with (1/V)int|u'|^2 = noise_rms^2.
    """
    gamma = 2.0 * math.pi / lz
    u = laminar_field(nx, ny, nz)
    if ny < 5:
        raise ValueError("streak_roll_field needs Ny >= 5")
    # cos(gamma z) -> stored m_z=1 coefficient 1/2 ; sin(gamma z) -> -i/2.
    one_m_y2 = np.array([0.5, 0.0, -0.5])                   # 1 - y^2
    q = np.array([3.0 / 8.0, 0.0, -0.5, 0.0, 1.0 / 8.0])    # (1 - y^2)^2
    y1my2 = np.array([0.0, 0.25, 0.0, -0.25])                # y (1 - y^2)
    a_roll = roll_amp / gamma
    u[1, 0, 1, : len(q)] += a_roll * gamma * q * 0.5                 # v = A g (1-y^2)^2 cos
    u[2, 0, 1, : len(y1my2)] += 4.0 * a_roll * y1my2 * (-0.5j)       # w = 4A y(1-y^2) sin
    u[0, 0, 1, : len(one_m_y2)] += -streak_amp * one_m_y2 * 0.5      # u = -B (1-y^2) cos
    noise = perturbation(nx, ny, nz, lx, lz, seed, energy=0.5 * noise_rms ** 2)
    return hermitian_project(u + noise)


def random_admissible(nx: int, ny: int, nz: int, lx: float, lz: float, seed: int,
                      scale: float = 1.0) -> np.ndarray:
    """A random divergence-free, no-slip field (no laminar part), unit-ish size.

    Used as Jacobian directions: it vanishes at the walls like every JVP input.
    """
    return perturbation(nx, ny, nz, lx, lz, seed, energy=0.5 * scale ** 2)


def random_spectral(nx: int, ny: int, nz: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A random canonical field with no constraints besides Hermitian/Nyquist.

    Used for adjoint (dot-product) tests and raw RHS vectors of the implicit
    solve, where admissibility is not required.
    """
    rng = np.random.default_rng(seed)
    shape = (3, nx, nz // 2 + 1, ny)
    a = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale
    return hermitian_project(a)


def regrid(a: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """The canonical field a on another grid: Fourier modes and Chebyshev
    coefficients present on both grids are copied, the others are zero
    (spectral interpolation by zero padding, or truncation). The result has
    zero Nyquist entries and keeps a's Hermitian m_z = 0 plane."""
    a = np.asarray(a)
    _, ax, azh, ay = a.shape
    out = np.zeros((3, nx, nz // 2 + 1, ny), dtype=np.complex128)
    hx = min(ax, nx) // 2          # |m_x| < hx on both grids
    hz = min(azh - 1, nz // 2)     # m_z < hz on both grids
    n = min(ay, ny)
    for m in range(-(hx - 1), hx):
        out[:, m % nx, :hz, :n] = a[:, m % ax, :hz, :n]
    return hermitian_project(out)


def embed_periodic(a: np.ndarray, fx: int, fz: int) -> np.ndarray:
    """The canonical field a of an Lx x Lz box as a field of the fx Lx x fz Lz
    box (integers fx, fz >= 1): the same function of (x, y, z), periodic
    extension, so mode (m_x, m_z) moves to (fx m_x, fz m_z) of an
    (fx nx) x (fz nz) grid and every other mode is zero. An equilibrium of the
    small box is one of the large box, in its subspace of fields invariant
    under the translations by Lx and Lz."""
    a = np.asarray(a)
    _, nxs, nzhs, ny = a.shape
    nxb, nzb = fx * nxs, fz * 2 * (nzhs - 1)
    out = np.zeros((3, nxb, nzb // 2 + 1, ny), dtype=np.complex128)
    for i in range(nxs):
        if i == nxs // 2:
            continue  # Nyquist: zero in canonical fields
        m = i if i < nxs // 2 else i - nxs
        for j in range(nzhs - 1):
            out[:, (fx * m) % nxb, fz * j, :] = a[:, i, j, :]
    return out
