"""The multi-step time-integration operator (test infrastructure only).

Sec. 2, eqs. Gstokes and Gint: G^Stokes_T = B_T - I takes one BEFE step of
length T, G^int_T = (B_dt)^{T/dt} - I takes T/dt steps of a small dt, so that
it approximates the flow map of the Navier-Stokes equations over time T.
The paper allows any scheme for B_dt in G^int; the reading here is BEFE (the
same Phi_dt as the Stokes operator, at the small dt), and the residual is
scaled by 1/T like the Stokes residual r = (Phi_T(U) - U)/T:

    r^int(U) = (Phi_dt^n(U) - U) / (n dt),   n = T / dt.

Its Jacobian follows from the chain rule along the trajectory
U_k = Phi_dt^k(U): J v = (J_Phi(U_{n-1}) ... J_Phi(U_0) v - v) / (n dt).

Pins (tests/test_oracle_gint.py): the laminar flow is a root; n = 1 is the
Stokes residual; the JVP matches central differences with an O(h^2) error
(which a Jacobian taken at the wrong trajectory point fails); halving dt at
fixed T halves the distance between the n-step and 2n-step maps (BEFE is
first-order accurate in time). SBDF2 (below): the laminar flow is a root,
one step is a BEFE step of tau, the JVP matches central differences, and
about U = 0 with walls at rest (where the linearised product vanishes along
the whole trajectory) an eigenvector of one
BEFE step with eigenvalue mu is one of the n-step map with the value d_n of
the scalar recurrence d_{k+1} = mu (4 d_k - d_{k-1}) / 3, d_{-1} = d_0 = 1.
"""
from __future__ import annotations

import numpy as np

from . import krylov, pack


def trajectory(befe, u: np.ndarray, n: int):
    """[U_0, ..., U_n] with U_{k+1} = Phi_dt(U_k)."""
    traj = [u]
    for _ in range(n):
        traj.append(befe.phi(traj[-1]))
    return traj


def residual(befe, u: np.ndarray, n: int) -> np.ndarray:
    return (trajectory(befe, u, n)[-1] - u) / (n * befe.dt)


def jvp(befe, u: np.ndarray, du: np.ndarray, n: int) -> np.ndarray:
    traj = trajectory(befe, u, n - 1)
    v = du
    for k in range(n):
        v = befe.jvp(traj[k], v, "phi")
    return (v - du) / (n * befe.dt)


# ---- SBDF2 as the integrator ------------------------------------------------------
# Second-order semi-implicit backward differences with the nonlinear term
# extrapolated, for du/dt = L u + N(u) with time step h:
#   (3 u_{k+1} - 4 u_k + u_{k-1}) / (2 h) = L u_{k+1} + 2 N(u_k) - N(u_{k-1}),
# i.e. with tau = 2 h / 3 one constrained solve of (I - tau L) per step:
#   u_{k+1} = (I - tau L)^{-1} [ (4 u_k - u_{k-1}) / 3 + tau (2 N(u_k) - N(u_{k-1})) ].
# `befe` is built with dt = tau (its solver is that of (I - tau L)). The start
# u_{-1} = u_0 = U makes the first step a BEFE step of tau. r = (u_n - U) / T
# with T = n h = 1.5 n tau.

def sbdf2_trajectory(befe, u: np.ndarray, n: int):
    """[U_0, ..., U_n] of the SBDF2 steps from U_{-1} = U_0 = u."""
    traj = [u]
    prev, cur = u, u
    n_prev = befe.nonlinear(u)
    for k in range(n):
        n_cur = befe.nonlinear(cur)
        if k == 0:
            n_prev = n_cur
        rhs = ((4.0 * cur - prev) / 3.0) / befe.dt + 2.0 * n_cur - n_prev
        nxt = befe.solver.solve(rhs, befe.wall_upper, befe.wall_lower)
        prev, cur, n_prev = cur, nxt, n_cur
        traj.append(cur)
    return traj


def sbdf2_residual(befe, u: np.ndarray, n: int) -> np.ndarray:
    return (sbdf2_trajectory(befe, u, n)[-1] - u) / (1.5 * n * befe.dt)


def sbdf2_jvp(befe, u: np.ndarray, du: np.ndarray, n: int) -> np.ndarray:
    """Chain rule of the SBDF2 steps along the trajectory (du_{-1} = du_0 = du,
    homogeneous walls)."""
    traj = sbdf2_trajectory(befe, u, n - 1)
    prev, cur = du, du
    l_prev = None
    for k in range(n):
        l_cur = befe.linearised_nonlinear(traj[k], cur)
        if k == 0:
            l_prev = l_cur
        rhs = ((4.0 * cur - prev) / 3.0) / befe.dt + 2.0 * l_cur - l_prev
        prev, cur, l_prev = cur, befe.solver.solve(rhs), l_cur
    return (cur - du) / (1.5 * n * befe.dt)


def newton_hook_gint(befe, U0_canonical: np.ndarray, n: int, tol: float, max_newton: int,
                     kmax: int, rtol: float, sbdf2: bool = False, **hook):
    """Trust-region Newton-GMRES (krylov.newton_hook) on r^int, packed vectors;
    BEFE steps of befe.dt, or SBDF2 steps with implicit step befe.dt."""
    g = befe.g
    res_f, jvp_f = (sbdf2_residual, sbdf2_jvp) if sbdf2 else (residual, jvp)

    def res(x):
        return pack.pack(res_f(befe, pack.unpack(x, g), n), g)

    def jv(x, dx):
        return pack.pack(jvp_f(befe, pack.unpack(x, g), pack.unpack(dx, g), n), g)

    def norm(rx):
        return befe.norm_l2(pack.unpack(rx, g))

    x, rep = krylov.newton_hook(res, jv, norm, pack.pack(U0_canonical, g), tol, max_newton,
                                kmax, rtol, **hook)
    return pack.unpack(x, g), rep
