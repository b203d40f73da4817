"""Chebyshev tools in the wall-normal direction (test infrastructure only).

Sec. 3.2: the wall-normal direction is represented by Chebyshev polynomials on
a Chebyshev (Gauss-Lobatto) grid, y_j = cos(pi j / N), j = 0..N. Conventions
(the paper is silent): T_n(cos t) = cos(n t); coefficients a_0..a_N.

Pins (tests/test_oracle_transforms.py): synthesis against
numpy.polynomial.chebyshev.chebval, analysis as the exact inverse of synthesis,
the derivative against chebder, the Gram matrix against Gauss-Legendre
quadrature of products of Chebyshev polynomials.
"""
from __future__ import annotations

import numpy as np


def points(N: int) -> np.ndarray:
    """Gauss-Lobatto points y_j = cos(pi j / N)."""
    j = np.arange(N + 1)
    return np.cos(np.pi * j / N)


def synthesis(N: int) -> np.ndarray:
    """T[j, n] = T_n(y_j): coefficients -> values at the Gauss-Lobatto points."""
    j = np.arange(N + 1)[:, None]
    n = np.arange(N + 1)[None, :]
    return np.cos(np.pi * j * n / N)


def analysis(N: int) -> np.ndarray:
    """Exact inverse of synthesis on polynomials of degree <= N.

    a_n = 2 / (N cb_n) * sum_j f_j T_n(y_j) / cb_j with cb_0 = cb_N = 2, else 1.
    """
    cb = np.ones(N + 1)
    cb[0] = cb[N] = 2.0
    n = np.arange(N + 1)[:, None]
    j = np.arange(N + 1)[None, :]
    return (2.0 / N) * np.cos(np.pi * n * j / N) / (cb[:, None] * cb[None, :])


def derivative(N: int) -> np.ndarray:
    """Coefficient-space d/dy: (D a)_n = (2 / c_n) sum_{m > n, m + n odd} m a_m.

    c_0 = 2, c_n = 1 otherwise. Follows from T_m' expressed in Chebyshev
    polynomials of lower degree.
    """
    D = np.zeros((N + 1, N + 1))
    for n in range(N + 1):
        for m in range(n + 1, N + 1):
            if (m + n) % 2 == 1:
                D[n, m] = 2.0 * m / (2.0 if n == 0 else 1.0)
    return D


def gram(N: int) -> np.ndarray:
    """G[n, m] = integral_{-1}^{1} T_n T_m dy.

    T_n T_m = (T_{n+m} + T_{|n-m|}) / 2 and integral T_k = 2 / (1 - k^2) for
    even k, 0 for odd k.
    """
    G = np.zeros((N + 1, N + 1))
    for n in range(N + 1):
        for m in range(N + 1):
            if (n + m) % 2 == 0:
                G[n, m] = 1.0 / (1.0 - (n + m) ** 2) + 1.0 / (1.0 - (n - m) ** 2)
    return G


def apply_y(M: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Apply an (N+1) x (N+1) matrix along the last axis of a."""
    return np.einsum("jn,...n->...j", M, a)


def values_at_walls(N: int):
    """Rows giving a(1) = sum a_n and a(-1) = sum (-1)^n a_n."""
    n = np.arange(N + 1)
    return np.ones(N + 1), (-1.0) ** n
