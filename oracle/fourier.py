"""Fourier transforms in the periodic directions (test infrastructure only).

Sec. 3.2: the two periodic directions are Fourier series; derivatives are
taken in Fourier space and products formed pointwise on a physical grid
(pseudospectral method). The physical grid is padded by 3/2 in x and z so
that the quadratic product is alias free for all retained modes (the paper
does not state its dealiasing; the 3/2 rule is the reading used here).

Conventions: u(x, z) = sum over all (m_x, m_z) of u_m exp(i(alpha m_x x +
gamma m_z z)); the forward transform carries the 1/(Px Pz) factor. numpy's
pocketfft (irfft2 / rfft2, norm="forward") is the library primitive.

Pins (tests/test_oracle_transforms.py): round trip, a single-mode closed form
and the brute-force O(N^4) product of the dealiasing test.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def to_physical(a: np.ndarray, g: Grid) -> np.ndarray:
    """Spectral y-valued array [..., Nx, Nz/2+1, Ny] -> physical [..., Px, Pz, Ny]."""
    lead = a.shape[:-3]
    A = np.zeros(lead + (g.px, g.pz // 2 + 1, g.ny), dtype=np.complex128)
    valid = g.valid()
    pidx = g.padded_x_index()
    for i in range(g.nx):
        for j in range(g.nzh):
            if valid[i, j]:
                A[..., pidx[i], j, :] = a[..., i, j, :]
    n = len(lead)
    return np.fft.irfft2(A, s=(g.px, g.pz), axes=(n, n + 1), norm="forward")


def to_spectral(p: np.ndarray, g: Grid) -> np.ndarray:
    """Physical [..., Px, Pz, Ny] -> truncated spectral [..., Nx, Nz/2+1, Ny]."""
    lead = p.shape[:-3]
    n = len(lead)
    B = np.fft.rfft2(p, axes=(n, n + 1), norm="forward")
    out = np.zeros(lead + (g.nx, g.nzh, g.ny), dtype=np.complex128)
    valid = g.valid()
    pidx = g.padded_x_index()
    for i in range(g.nx):
        for j in range(g.nzh):
            if valid[i, j]:
                out[..., i, j, :] = B[..., pidx[i], j, :]
    return out


def physical_grid(g: Grid):
    """Padded physical x and z coordinates."""
    x = np.arange(g.px) * g.lx / g.px
    z = np.arange(g.pz) * g.lz / g.pz
    return x, z
