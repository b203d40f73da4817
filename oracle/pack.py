"""Canonical complex layout <-> packed real vector (test infrastructure only).

The packed vector lists each real degree of freedom once: for every velocity
component c and Chebyshev index n, the (0,0) mode (real part), then the
m_z = 0 modes with m_x = 1..Nx/2-1 as (Re, Im) pairs, then for m_z =
1..Nz/2-1 every non-Nyquist m_x in FFT order as (Re, Im). Its length is
3 Ny (Nx-1)(Nz-1). The Euclidean product of packed vectors is the inner
product GMRES and autograd use.

Pins (tests/test_oracle_transforms.py): pack(unpack(x)) = x; the packed
product equals the Parseval-weighted canonical product with the (0,0) mode
counted once.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def _mode_list(g: Grid):
    lst = [(0, 0, False)]
    for i in range(1, g.nx // 2):
        lst.append((i, 0, True))
    for j in range(1, g.nz // 2):
        for i in range(g.nx):
            if i == g.nx // 2:
                continue
            lst.append((i, j, True))
    return lst


def packed_length(g: Grid) -> int:
    return 3 * g.ny * (g.nx - 1) * (g.nz - 1)


def pack(a: np.ndarray, g: Grid) -> np.ndarray:
    out = []
    modes = _mode_list(g)
    for c in range(3):
        for n in range(g.ny):
            for (i, j, cplx) in modes:
                v = a[c, i, j, n]
                out.append(v.real)
                if cplx:
                    out.append(v.imag)
    return np.array(out, dtype=np.float64)


def unpack(x: np.ndarray, g: Grid) -> np.ndarray:
    a = g.zeros()
    modes = _mode_list(g)
    k = 0
    for c in range(3):
        for n in range(g.ny):
            for (i, j, cplx) in modes:
                if cplx:
                    a[c, i, j, n] = x[k] + 1j * x[k + 1]
                    k += 2
                else:
                    a[c, i, j, n] = x[k]
                    k += 1
    for i in range(1, g.nx // 2):
        a[:, g.nx - i, 0, :] = np.conj(a[:, i, 0, :])
    return a


def packed_dot(a: np.ndarray, b: np.ndarray, g: Grid) -> float:
    """Packed Euclidean product evaluated on canonical arrays."""
    w = np.ones((g.nx, g.nzh))
    w[:, 0] = 0.5
    w[0, 0] = 1.0
    w[g.nx // 2, :] = 0.0
    w[:, g.nzh - 1] = 0.0
    return float(np.sum(w[None, :, :, None] * (a.conj() * b).real))
