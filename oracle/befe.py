"""Phi_dt, its residual, Jacobian-vector and vector-Jacobian products.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 2, eq. befe: B_dt = (I - dt L)^{-1} (I + dt N). With L = (1/Re) Lap and
the constraints folded into the implicit solve, one step is

    Phi_dt(u) = S(u/dt + N(u)),

where S solves (1/Re) Lap phi - phi/dt - grad p = -g with the wall velocities
as boundary values (oracle.stokes). The residual whose root is sought is
r = (Phi_dt(u) - u)/dt = G^Stokes_T / T with T = dt (Sec. 2, eq. Gstokes).

N(u) is the advective term (Sec. 2) in rotational form, N(u) = u x omega with
omega = curl u; the gradient part of (u.grad)u is a pressure gradient that the
implicit solve absorbs. It is formed pseudospectrally (Sec. 3.2): derivatives
in spectral space, values at the Gauss-Lobatto points in y, 3/2-padded FFTs in
x and z, the pointwise product, and the inverse path with truncation.

The Jacobian action (Sec. 2, after eq. factor2) replaces N by its
linearisation about U, N_U(du) = du x Omega + U x curl(du), and every
inhomogeneous boundary value by zero:

    J_Phi(U) du = S_0(du/dt + N_U(du)),   J_r(U) du = (J_Phi du - du)/dt.

The vector-Jacobian product is the adjoint of J_Phi in the packed Euclidean
inner product (oracle.pack). It is formed stage by stage with each stage's
explicit adjoint with respect to the inner product
<a, b> = sum over stored modes of w_m Re(conj a . b), w_m = 1 for m_z = 0 and
2 for m_z > 0 (Parseval weight), then converted to the packed product.

Pins (tests/test_oracle_befe.py): laminar Couette flow is a fixed point
(Sec. 3.1 U_lam = y; eq. befe); the increment identity B - I =
(I - dt L)^{-1} dt (L + N) (Sec. 2, eq. mycalc) with L+N formed without any
solve; the large-dt limit -L^{-1}(L+N) (eq. largedt); divergence and wall
values; the brute-force dealiased product; exactness of the central
difference for the quadratic map (eq. finitediff); translation and
reflection symmetries; adjoint dot-product identities and the dense
Jacobian transpose; the sign of N against the convective form -(u.grad)u
plus a gradient, and the curl of single-mode fields in closed form.
"""
from __future__ import annotations

import numpy as np

from . import cheb
from . import fourier
from .grid import Grid
from .stokes import StokesSolver


class Befe:
    def __init__(self, g: Grid, re: float, dt: float, wall_upper: float = 1.0,
                 wall_lower: float = -1.0, modes=None):
        self.g = g
        self.re = float(re)
        self.dt = float(dt)
        self.wall_upper = float(wall_upper)
        self.wall_lower = float(wall_lower)
        N = g.N
        self.T = cheb.synthesis(N)
        self.Tinv = cheb.analysis(N)
        self.D = cheb.derivative(N)
        self.G = cheb.gram(N)
        self.solver = StokesSolver(g, re, dt, modes)
        self.ikx = (1j * g.kx())[:, None, None]
        self.ikz = (1j * g.kz())[None, :, None]

    # ---- spectral building blocks -------------------------------------------------
    def dy(self, a):
        return cheb.apply_y(self.D, a)

    def curl(self, a):
        """omega = curl u in coefficient space: d/dx -> i k_x, d/dz -> i k_z."""
        u, v, w = a[0], a[1], a[2]
        return np.stack([self.dy(w) - self.ikz * v,
                         self.ikz * u - self.ikx * w,
                         self.ikx * v - self.dy(u)])

    def laplacian(self, a):
        k2 = -(self.ikx * self.ikx + self.ikz * self.ikz).real
        return cheb.apply_y(self.D @ self.D, a) - k2 * a

    def to_physical(self, a):
        """Coefficients -> values on the padded physical grid [.., Px, Pz, Ny]."""
        return fourier.to_physical(cheb.apply_y(self.T, a), self.g)

    def to_coefficients(self, p):
        """Physical values -> truncated spectral Chebyshev coefficients."""
        return cheb.apply_y(self.Tinv, fourier.to_spectral(p, self.g))

    # ---- the map ------------------------------------------------------------------------
    def nonlinear(self, u):
        """N(u) = u x curl(u), dealiased (coefficients)."""
        up = self.to_physical(u)
        wp = self.to_physical(self.curl(u))
        return self.to_coefficients(np.cross(up, wp, axis=0))

    def linearised_nonlinear(self, U, du):
        """N_U(du) = du x Omega + U x curl(du)."""
        Up = self.to_physical(U)
        Op = self.to_physical(self.curl(U))
        dp = self.to_physical(du)
        dwp = self.to_physical(self.curl(du))
        return self.to_coefficients(np.cross(dp, Op, axis=0) + np.cross(Up, dwp, axis=0))

    def phi(self, u):
        return self.solver.solve(u / self.dt + self.nonlinear(u),
                                 self.wall_upper, self.wall_lower)

    def residual(self, u):
        return (self.phi(u) - u) / self.dt

    def jvp(self, U, du, op: str = "phi"):
        out = self.solver.solve(du / self.dt + self.linearised_nonlinear(U, du))
        if op == "phi":
            return out
        return (out - du) / self.dt

    # ---- adjoint ---------------------------------------------------------------------------
    def solve_adjoint(self, w):
        """Adjoint of the homogeneous solve S_0 in the Parseval inner product
        (per mode the conjugate transpose, oracle.stokes)."""
        return self.solver.solve_adjoint(w)

    def curl_adjoint(self, a):
        ax, ay, az = a[0], a[1], a[2]
        DT = lambda b: cheb.apply_y(self.D.T, b)
        return np.stack([-self.ikz * ay - DT(az),
                         self.ikz * ax - self.ikx * az,
                         DT(ax) + self.ikx * ay])

    def physical_adjoint(self, p):
        """Adjoint of to_physical (coefficients -> physical values)."""
        g = self.g
        return cheb.apply_y(self.T.T, fourier.to_spectral(p, g)) * (g.px * g.pz)

    def coefficients_adjoint(self, a):
        """Adjoint of to_coefficients (physical values -> coefficients)."""
        g = self.g
        return fourier.to_physical(cheb.apply_y(self.Tinv.T, a), g) / (g.px * g.pz)

    def vjp_parseval(self, U, w):
        """J_Phi(U)^dagger w in the Parseval inner product."""
        a = self.solve_adjoint(w)
        npb = self.coefficients_adjoint(a)
        Up = self.to_physical(U)
        Op = self.to_physical(self.curl(U))
        d_phys = np.cross(Op, npb, axis=0)      # adjoint of du -> du x Omega
        w_phys = np.cross(npb, Up, axis=0)      # adjoint of dw -> U x dw
        return a / self.dt + self.physical_adjoint(d_phys) + \
            self.curl_adjoint(self.physical_adjoint(w_phys))

    def vjp(self, U, w, op: str = "phi"):
        """J^T w in the packed Euclidean inner product (canonical arrays)."""
        w2 = np.array(w, copy=True)
        w2[:, 0, 0, :] *= 2.0
        out = self.vjp_parseval(U, w2)
        out[:, 0, 0, :] *= 0.5
        if op == "phi":
            return out
        return (out - w) / self.dt

    # ---- norms ---------------------------------------------------------------------------
    def norm_l2(self, a) -> float:
        """Volume-normalised L2 norm sqrt((1/V) int |a|^2 dV) (Parseval + Gram)."""
        g = self.g
        wts = np.where(g.mz() == 0, 1.0, 2.0)[None, None, :, None]
        Ga = cheb.apply_y(self.G, a)
        s = np.sum(wts * (a.conj() * Ga).real)
        return float(np.sqrt(0.5 * s))

    def divergence(self, a):
        return self.ikx * a[0] + self.dy(a[1]) + self.ikz * a[2]

    def wall_values(self, a):
        top, bot = cheb.values_at_walls(self.g.N)
        return a @ top, a @ bot
