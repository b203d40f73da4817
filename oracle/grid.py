"""Mode bookkeeping for the canonical layout (test infrastructure only).

Canonical spectral array: complex128 [3][Nx][Nz/2+1][Ny].
* axis 1: Fourier index i in x, m_x = i for i < Nx/2 and i - Nx otherwise;
  i = Nx/2 is the Nyquist mode and is always zero;
* axis 2: m_z = 0..Nz/2; m_z = Nz/2 is the Nyquist mode and is always zero;
* axis 3: Chebyshev coefficient n = 0..N, N = Ny - 1 (or, for "y-valued"
  arrays, the Gauss-Lobatto point index j, y_j = cos(pi j / N)).

The box is [0, Lx) x [-1, 1] x [0, Lz), alpha = 2 pi / Lx, gamma = 2 pi / Lz;
Sec. 3.3 uses Lx = 2 pi / 1.14, Lz = 2 pi / 2.5. The grid numbers follow the
paper's (M_x, M_y, M_z) triplets read as: unpadded Fourier sizes in x and z,
Gauss-Lobatto point count in y; products are formed on the 3/2-padded grid.
Pins: tests/test_oracle_transforms.py (mode bookkeeping is exercised by the
FFT round trip and the brute-force product).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float

    def __post_init__(self):
        if self.nx < 4 or self.nx % 2 or self.nz < 4 or self.nz % 2:
            raise ValueError("nx, nz must be even and >= 4")
        if self.ny < 5:
            raise ValueError("ny must be >= 5")

    @property
    def N(self) -> int:
        return self.ny - 1

    @property
    def nzh(self) -> int:
        return self.nz // 2 + 1

    @property
    def px(self) -> int:
        return 3 * self.nx // 2

    @property
    def pz(self) -> int:
        return 3 * self.nz // 2

    @property
    def alpha(self) -> float:
        return 2.0 * math.pi / self.lx

    @property
    def gamma(self) -> float:
        return 2.0 * math.pi / self.lz

    @property
    def shape(self):
        return (3, self.nx, self.nzh, self.ny)

    def mx(self) -> np.ndarray:
        return np.array([i if i < self.nx // 2 else i - self.nx for i in range(self.nx)],
                        dtype=np.int64)

    def mz(self) -> np.ndarray:
        return np.arange(self.nzh, dtype=np.int64)

    def kx(self) -> np.ndarray:
        return self.alpha * self.mx().astype(np.float64)

    def kz(self) -> np.ndarray:
        return self.gamma * self.mz().astype(np.float64)

    def valid(self) -> np.ndarray:
        """[Nx, Nz/2+1] mask of kept modes (Nyquist excluded)."""
        m = np.ones((self.nx, self.nzh), dtype=bool)
        m[self.nx // 2, :] = False
        m[:, self.nzh - 1] = False
        return m

    def padded_x_index(self) -> np.ndarray:
        """Index of each canonical m_x in the padded x spectrum of length Px."""
        return np.mod(self.mx(), self.px)

    def zeros(self) -> np.ndarray:
        return np.zeros(self.shape, dtype=np.complex128)
