"""The BEFE step with the laminar advection in the implicit operator.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 3.6 proposes, as the most promising remedy for the large Krylov counts at
high Re, moving the linearisation of the advection about the laminar flow,
(U_lam . grad) u + (u . grad) U_lam, from N into L. With U_lam = y e_x this
linear operator is, per Fourier mode (k_x = alpha m_x),

    M u = -( i k_x y u + v,  i k_x y v,  i k_x y w )

(convective form; it differs from the rotational U_lam x omega(u) +
u x Omega_lam by the gradient of y u, which the pressure absorbs). The step
becomes

    (I - dt (L + M)) Phi~(U) = U + dt (N(U) - M U)

with the same constraints, so the steady equation L U + N(U) = 0, and with it
every root, is unchanged (M U_lam = 0). Multiplication by y acts on Chebyshev
coefficients as y T_0 = T_1, y T_n = (T_{n-1} + T_{n+1})/2; in the tau rows
(n <= N-2) only coefficients up to N-1 enter, so nothing is truncated. Each
mode's system is the Stokes tau system of stokes.mode_matrix plus these
terms, solved densely with extended-precision refinement. The mean mode has
k_x = 0 and v = 0, so its problem is unchanged.

Pins (tests/test_oracle_advect.py): the coefficient-space multiplication by y
against numpy's Chebyshev chebmulx; M against the same operator evaluated on
the physical grid; the laminar flow is a fixed point; the increment identity
Phi~(u) - u = S~_0[L u + N(u)] (S~_0 the augmented solve with no-slip walls);
for k_x = 0 the lift-up coupling decouples as the plain Stokes solve for
(v, w, p) followed by the x-momentum solve with right-hand side g_u - v.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .befe import Befe
from .grid import Grid
from .stokes import StokesSolver, _refined_solve, mean_matrix, mode_matrix, mode_rhs


def y_matrix(N: int) -> np.ndarray:
    """(N+1) x (N+1): Chebyshev coefficients of y p(y) from those of p (the
    T_{N+1} part of y T_N dropped)."""
    Y = np.zeros((N + 1, N + 1))
    Y[1, 0] = 1.0
    for n in range(1, N + 1):
        Y[n - 1, n] += 0.5
        if n + 1 <= N:
            Y[n + 1, n] += 0.5
    return Y


def laminar_advection(g: Grid, a: np.ndarray) -> np.ndarray:
    """M a for a canonical field a (coefficients)."""
    Y = y_matrix(g.N)
    ikx = (1j * g.kx())[:, None, None]
    ya = np.einsum("mn,cijn->cijm", Y, a)
    out = -(ikx[None] * ya)
    out[0] -= a[1]
    return out


def mode_matrix_adv(N: int, kx: float, kz: float, re: float, inv_dt: float) -> np.ndarray:
    """stokes.mode_matrix with M added to the three momentum blocks."""
    A = mode_matrix(N, kx, kz, re, inv_dt)
    n1 = N + 1
    Y = y_matrix(N)
    U, V, W = 0, n1, 2 * n1
    r = 0
    for off in (U, V, W):
        for n in range(N - 1):
            A[r + n, off:off + n1] -= 1j * kx * Y[n]
        r += N - 1
    for n in range(N - 1):              # -v in the x-momentum rows
        A[n, V + n] -= 1.0
    return A


class AdvectedSolver(StokesSolver):
    """StokesSolver with the laminar advection in the implicit operator."""

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
                A = mode_matrix_adv(N, kx[i], kz[j], self.re, self.inv_dt)
            self._fact[(i, j)] = (A, sla.lu_factor(A))


class AdvBefe(Befe):
    """Phi~(U) = (I - dt(L + M))^{-1} (U + dt (N(U) - M U)) and its Jacobian."""

    def __init__(self, g: Grid, re: float, dt: float, wall_upper: float = 1.0,
                 wall_lower: float = -1.0, modes=None):
        super().__init__(g, re, dt, wall_upper, wall_lower, modes=[(0, 0)])
        self.solver = AdvectedSolver(g, re, dt, modes)

    def phi(self, u):
        rhs = u / self.dt + self.nonlinear(u) - laminar_advection(self.g, u)
        return self.solver.solve(rhs, self.wall_upper, self.wall_lower)

    def jvp(self, U, du, op: str = "phi"):
        rhs = du / self.dt + self.linearised_nonlinear(U, du) - laminar_advection(self.g, du)
        out = self.solver.solve(rhs)
        if op == "phi":
            return out
        return (out - du) / self.dt

    def vjp(self, U, w, op: str = "phi"):
        raise NotImplementedError("the adjoint of the advected step is not provided")
