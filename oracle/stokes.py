"""The implicit half of the BEFE step: (I - dt L)^{-1} with its constraints.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 2 (after eq. befe) places the boundary conditions, incompressibility and
the pressure inside the implicit operator (I - dt L)^{-1}; Sec. 3.2 requires
the inversion to be exact (direct, not iterative) and the result divergence
free to machine accuracy. For each Fourier mode (m_x, m_z) with
k_x = alpha m_x, k_z = gamma m_z, k^2 = k_x^2 + k_z^2, the discrete problem
solved here is the coupled Chebyshev-tau Stokes system for the coefficients of
(u, v, w, p), each a polynomial of degree <= N:

  (1/Re)(D^2 - k^2) u - u/dt - i k_x p = -g_u     on T_0 .. T_{N-2}
  (1/Re)(D^2 - k^2) v - v/dt - D p     = -g_v     on T_0 .. T_{N-2}
  (1/Re)(D^2 - k^2) w - w/dt - i k_z p = -g_w     on T_0 .. T_{N-2}
  u(+-1) = v(+-1) = w(+-1) = 0
  i k_x u + D v + i k_z w = 0                      on T_0 .. T_N

i.e. 4N+4 equations for 4N+4 unknowns. Reading of the paper: the momentum
equations are imposed on all but the two highest Chebyshev coefficients (the
standard tau method; the two highest coefficients of g are discarded), and the
divergence vanishes identically, which is what "divergence free to machine
accuracy" asks of the influence-matrix method.

The mean mode (0,0) carries no pressure gradient along the walls (plane
Couette flow, Sec. 3.1): u and w solve scalar Dirichlet Helmholtz problems
(1/Re) D^2 u - u/dt = -g on T_0..T_{N-2} with u(1) = wall_upper, u(-1) =
wall_lower for the full step (0 for linearised and adjoint steps), and v = 0.

Each system is assembled densely and solved by LU, followed by two steps of
iterative refinement whose residuals are computed in extended precision
(numpy clongdouble); all matrix entries are exact in fp64, so the refined
result is the fp64 rounding of the exact solution up to a small multiple of
the unit round-off.

Pins (tests/test_oracle_stokes.py): manufactured polynomial solutions that
satisfy the tau system exactly, the closed-form solution of the (0,0)
Helmholtz problem, analytic Stokes eigenvalues of the channel (Dirichlet
Laplacian families and the v-family roots of s tan s = -k tanh k and
s cot s = k coth k), divergence and wall values of every solution.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import cheb
from .grid import Grid


def mode_matrix(N: int, kx: float, kz: float, re: float, inv_dt: float) -> np.ndarray:
    """Dense (4N+4) x (4N+4) tau system for one mode (k != 0).

    Unknown order: u_0..u_N, v_0..v_N, w_0..w_N, p_0..p_N.
    Row order: x-momentum (N-1 rows), y-momentum, z-momentum, six wall rows
    (u(1), u(-1), v(1), v(-1), w(1), w(-1)), continuity (N+1 rows).
    """
    n1 = N + 1
    D = cheb.derivative(N)
    D2 = D @ D
    k2 = kx * kx + kz * kz
    H = D2 / re - (k2 / re + inv_dt) * np.eye(n1)
    A = np.zeros((4 * n1, 4 * n1), dtype=np.complex128)
    U, V, W, P = 0, n1, 2 * n1, 3 * n1
    r = 0
    for n in range(N - 1):              # x-momentum
        A[r, U:U + n1] = H[n]
        A[r, P + n] = -1j * kx
        r += 1
    for n in range(N - 1):              # y-momentum
        A[r, V:V + n1] = H[n]
        A[r, P:P + n1] = -D[n]
        r += 1
    for n in range(N - 1):              # z-momentum
        A[r, W:W + n1] = H[n]
        A[r, P + n] = -1j * kz
        r += 1
    top, bot = cheb.values_at_walls(N)
    for off in (U, V, W):               # no-slip walls
        A[r, off:off + n1] = top
        r += 1
        A[r, off:off + n1] = bot
        r += 1
    for n in range(n1):                 # continuity on every coefficient
        A[r, U + n] = 1j * kx
        A[r, V:V + n1] = D[n]
        A[r, W + n] = 1j * kz
        r += 1
    assert r == 4 * n1
    return A


def mode_rhs(N: int, g: np.ndarray) -> np.ndarray:
    """Right-hand side for mode_matrix from g = [g_u, g_v, g_w] (3, N+1)."""
    n1 = N + 1
    b = np.zeros(4 * n1, dtype=np.complex128)
    b[0:N - 1] = -g[0, :N - 1]
    b[N - 1:2 * N - 2] = -g[1, :N - 1]
    b[2 * N - 2:3 * N - 3] = -g[2, :N - 1]
    return b


def mean_matrix(N: int, re: float, inv_dt: float) -> np.ndarray:
    """(N+1) x (N+1) Dirichlet Helmholtz tau matrix of the (0,0) mode."""
    D = cheb.derivative(N)
    H = (D @ D) / re - inv_dt * np.eye(N + 1)
    A = np.zeros((N + 1, N + 1))
    A[:N - 1] = H[:N - 1]
    top, bot = cheb.values_at_walls(N)
    A[N - 1] = top
    A[N] = bot
    return A


def _refined_solve(A: np.ndarray, lu, b: np.ndarray, steps: int = 2) -> np.ndarray:
    x = sla.lu_solve(lu, b)
    Ae = A.astype(np.clongdouble if np.iscomplexobj(A) else np.longdouble)
    for _ in range(steps):
        xe = x.astype(Ae.dtype)
        r = b.astype(Ae.dtype) - Ae @ xe
        dx = sla.lu_solve(lu, r.astype(b.dtype if np.iscomplexobj(b) else np.float64))
        x = (xe + dx.astype(Ae.dtype)).astype(x.dtype)
    return x


def _refined_solve_adjoint(A: np.ndarray, lu, b: np.ndarray, steps: int = 2) -> np.ndarray:
    """x with A^H x = b, from the LU factors of A, refined like _refined_solve."""
    cplx = np.iscomplexobj(A)
    x = sla.lu_solve(lu, b, trans=2 if cplx else 1)
    AH = A.conj().T.astype(np.clongdouble if cplx else np.longdouble)
    for _ in range(steps):
        xe = x.astype(AH.dtype)
        r = b.astype(AH.dtype) - AH @ xe
        dx = sla.lu_solve(lu, r.astype(np.complex128 if cplx else np.float64),
                          trans=2 if cplx else 1)
        x = (xe + dx.astype(AH.dtype)).astype(x.dtype)
    return x


class StokesSolver:
    """Per-mode dense factorisations of the implicit BEFE operator.

    solve(g, wall_upper, wall_lower) returns the velocity coefficients phi that
    solve the tau system above with right-hand side g (canonical layout). The
    factorisations depend only on (grid, Re, dt) and are cached per mode.
    ``modes`` restricts the solver to a subset of (i, j) canonical indices
    (other modes return zero), which lets parity tests sample large grids.
    """

    def __init__(self, g: Grid, re: float, dt: float, modes=None):
        self.g = g
        self.re = float(re)
        self.dt = float(dt)
        self.inv_dt = 0.0 if np.isinf(dt) else 1.0 / float(dt)
        N = g.N
        valid = g.valid()
        if modes is None:
            modes = [(i, j) for i in range(g.nx) for j in range(g.nzh) if valid[i, j]]
        self.modes = [tuple(m) for m in modes if valid[m[0], m[1]]]
        kx, kz = g.kx(), g.kz()
        self._fact = {}
        for (i, j) in self.modes:
            if i == 0 and j == 0:
                A = mean_matrix(N, self.re, self.inv_dt)
            else:
                A = mode_matrix(N, kx[i], kz[j], self.re, self.inv_dt)
            self._fact[(i, j)] = (A, sla.lu_factor(A))

    def solve(self, gfield: np.ndarray, wall_upper: float = 0.0,
              wall_lower: float = 0.0) -> np.ndarray:
        g = self.g
        N = g.N
        out = g.zeros()
        for (i, j) in self.modes:
            A, lu = self._fact[(i, j)]
            if i == 0 and j == 0:
                for c, (bt, bb) in ((0, (wall_upper, wall_lower)), (2, (0.0, 0.0))):
                    b = np.zeros(N + 1)
                    b[:N - 1] = -gfield[c, 0, 0, :N - 1].real
                    b[N - 1] = bt
                    b[N] = bb
                    out[c, 0, 0] = _refined_solve(A, lu, b)
                continue
            x = _refined_solve(A, lu, mode_rhs(N, gfield[:, i, j, :]))
            out[0, i, j] = x[0:N + 1]
            out[1, i, j] = x[N + 1:2 * N + 2]
            out[2, i, j] = x[2 * N + 2:3 * N + 3]
        return out

    def pressure(self, gfield: np.ndarray, i: int, j: int) -> np.ndarray:
        """Pressure coefficients of mode (i, j) != (0,0) for right-hand side g."""
        A, lu = self._fact[(i, j)]
        N = self.g.N
        x = _refined_solve(A, lu, mode_rhs(N, gfield[:, i, j, :]))
        return x[3 * N + 3:]

    def solve_adjoint(self, w: np.ndarray) -> np.ndarray:
        """Conjugate transpose of the homogeneous solve g -> phi, mode by mode.

        For a mode k != 0 the solve is S = P A^{-1} E, with E placing -g_c(n),
        n <= N-2, on the momentum rows and P keeping the velocity unknowns, so
        S^H w = E^H A^{-H} P^H w: one solve with A^H (the same LU factors) per
        mode. The (0,0) mode is real: S^T w = -(A^{-T} w) on n <= N-2.
        Pinned against the conjugate transpose of the explicit operators
        (mode_operator, mean_operator) in tests/test_oracle_stokes.py.
        """
        g = self.g
        N = g.N
        n1 = N + 1
        out = g.zeros()
        for (i, j) in self.modes:
            A, lu = self._fact[(i, j)]
            if i == 0 and j == 0:
                for c in (0, 2):
                    y = _refined_solve_adjoint(A, lu, np.ascontiguousarray(w[c, 0, 0].real))
                    out[c, 0, 0, :N - 1] = -y[:N - 1]
                continue
            b = np.zeros(4 * n1, dtype=np.complex128)
            b[:3 * n1] = w[:, i, j, :].reshape(-1)
            y = _refined_solve_adjoint(A, lu, b)
            for c in range(3):
                out[c, i, j, :N - 1] = -y[c * (N - 1):(c + 1) * (N - 1)]
        return out

    def mode_operator(self, i: int, j: int) -> np.ndarray:
        """Dense 3(N+1) x 3(N+1) complex map g -> phi for one mode (k != 0).

        Used by the adjoint (its conjugate transpose) and by spectra tests.
        """
        N = self.g.N
        n1 = N + 1
        A, lu = self._fact[(i, j)]
        S = np.zeros((3 * n1, 3 * n1), dtype=np.complex128)
        for col in range(3 * n1):
            gg = np.zeros((3, n1), dtype=np.complex128)
            gg[col // n1, col % n1] = 1.0
            x = _refined_solve(A, lu, mode_rhs(N, gg))
            S[:, col] = x[:3 * n1]
        return S

    def mean_operator(self) -> np.ndarray:
        """(N+1) x (N+1) real map g -> u of the (0,0) mode, homogeneous walls."""
        N = self.g.N
        A, lu = self._fact[(0, 0)]
        S = np.zeros((N + 1, N + 1))
        for col in range(N - 1):
            b = np.zeros(N + 1)
            b[col] = -1.0
            S[:, col] = _refined_solve(A, lu, b)
        return S
