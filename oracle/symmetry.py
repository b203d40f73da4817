"""The shift-reflect symmetry subspace of plane Couette equilibria (test
infrastructure only).

Sec. 3.3 computes EQ1, which is invariant under the group S = {1, s1, s2, s3}
of the Couette symmetries (Gibson, Halcrow & Cvitanovic 2008):

    s1 [u, v, w](x, y, z) = [u, v, -w](x + Lx/2, y, -z),
    s2 [u, v, w](x, y, z) = [-u, -v, w](-x + Lx/2, -y, z + Lz/2),
    s3 = s1 s2.

Phi commutes with each of them (they are symmetries of the equations and the
walls), so the S-invariant fields form an invariant subspace in which Newton
solves can be confined; it excludes the translation directions d/dx U and
d/dz U of an invariant state. The projector P = (1 + s1 + s2 + s3)/4 is
composed here from the elementary operations on coefficients: translation by
(sx, sz) multiplies mode (m_x, m_z) by exp(i (k_x sx + k_z sz)); z -> -z maps
mode m_x to the conjugate of mode -m_x (w negated); (x, y) -> (-x, -y) maps
mode m_x to mode -m_x with T_n(-y) = (-1)^n T_n(y) (u, v negated).

Pins (tests/test_oracle_symmetry.py): P is idempotent, its image is invariant
under s1 and s2 separately, s1 and s2 are involutions, and Phi maps invariant
fields to invariant fields.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def _neg(g: Grid):
    return np.array([(g.nx - i) % g.nx for i in range(g.nx)])


def translate(g: Grid, a: np.ndarray, sx: float, sz: float) -> np.ndarray:
    ph = np.exp(1j * (g.kx()[:, None, None] * sx + g.kz()[None, :, None] * sz))
    return a * ph[None]


def reflect_z(g: Grid, a: np.ndarray) -> np.ndarray:
    out = np.conj(a[:, _neg(g)])
    out[2] *= -1
    return out


def rotate_xy(g: Grid, a: np.ndarray) -> np.ndarray:
    out = a[:, _neg(g)] * ((-1.0) ** np.arange(g.ny))
    out[0] *= -1
    out[1] *= -1
    return out


def s1(g: Grid, a: np.ndarray) -> np.ndarray:
    # [u, v, -w](x + Lx/2, y, -z): reflect, then evaluate at x + Lx/2
    return translate(g, reflect_z(g, a), g.lx / 2, 0.0)


def s2(g: Grid, a: np.ndarray) -> np.ndarray:
    # [-u, -v, w](-x + Lx/2, -y, z + Lz/2) = rotation evaluated at x - Lx/2 ... :
    # f(-(x - Lx/2), -y, z + Lz/2), i.e. translate the rotated field by (-Lx/2, Lz/2)
    return translate(g, rotate_xy(g, a), -g.lx / 2, g.lz / 2)


def project(g: Grid, a: np.ndarray) -> np.ndarray:
    b = s2(g, a)
    return 0.25 * (a + s1(g, a) + b + s1(g, b))
