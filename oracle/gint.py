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
first-order accurate in time).
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


def newton_hook_gint(befe, U0_canonical: np.ndarray, n: int, tol: float, max_newton: int,
                     kmax: int, rtol: float, **hook):
    """Trust-region Newton-GMRES (krylov.newton_hook) on r^int, packed vectors."""
    g = befe.g

    def res(x):
        return pack.pack(residual(befe, pack.unpack(x, g), n), g)

    def jv(x, dx):
        return pack.pack(jvp(befe, pack.unpack(x, g), pack.unpack(dx, g), n), g)

    def norm(rx):
        return befe.norm_l2(pack.unpack(rx, g))

    x, rep = krylov.newton_hook(res, jv, norm, pack.pack(U0_canonical, g), tol, max_newton,
                                kmax, rtol, **hook)
    return pack.unpack(x, g), rep
