"""Spectra of the Newton operators' Jacobians (paper Sec. 3.5).

The distribution of the eigenvalues of G_U decides how fast GMRES converges
on eq. biglin. The paper forms the full Jacobian of G^Stokes_T = B_T - I or
G^int_T = (B_dt)^{T/dt} - I column by column, acting with the operator on
successive basis vectors, and computes its eigenvalues with LAPACK. Here the
columns are Jacobian actions of the plan on the GPU (the packed real basis
vectors, unpacked to canonical fields, one linearisation for all columns);
the eigenvalues are computed on the host (numpy, LAPACK geev). Only tiny
grids are practical: the matrix has packed_n^2 entries.

The plan's residual is r = G/T, so the Jacobian of G is T times the
Jacobian action of r (T = dt for the Stokes operator, nsteps * dt for the
time-integration operator).

Helpers for reading spectra: Beaume's rescaling of Stokes eigenvalues,
lambda -> (1 + T)/T lambda (eq. beaumescale), which tends to the spectrum of
L + N_U for small T and to that of -L^{-1}(L + N_U) for large T; and the two
statistics the paper quotes: the radius around -1 that contains a given
fraction of the spectrum, and the fraction whose real part lies within a
band around -1.
"""
from __future__ import annotations

import numpy as np

from ._lib import SP_OP_PHI, SP_OP_RESIDUAL


def jacobian_dense(plan, u, op: int = SP_OP_RESIDUAL, scale_to_g: bool = True) -> np.ndarray:
    """The dense Jacobian in the packed real basis: column i is the packed
    Jacobian action on the i-th unit vector. op = SP_OP_RESIDUAL gives the
    Jacobian of the plan's residual operator (times T if scale_to_g, i.e.
    the Jacobian of G = B - I); op = SP_OP_PHI gives that of one BEFE step."""
    plan.linearize(u)
    # rows of the device result are the columns of J
    J = np.ascontiguousarray(plan.jacobian_columns(op).cpu().numpy().T)
    if op == SP_OP_RESIDUAL and scale_to_g:
        step = 1.5 if getattr(plan, "scheme", 0) == 1 else 1.0  # SBDF2: time step 1.5 dt
        J *= plan.dt * getattr(plan, "nsteps", 1) * step
    return J


def eigenvalues(J: np.ndarray) -> np.ndarray:
    return np.linalg.eigvals(J)


def admissible_basis(J_phi: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """Orthonormal basis of the admissible (divergence-free, no-slip) fields:
    the range of the Jacobian of one BEFE step, which maps every packed vector
    into that subspace (from its SVD; rank by the relative tolerance)."""
    U, sv, _ = np.linalg.svd(J_phi)
    return U[:, : int(np.sum(sv > tol * sv[0]))]


def restrict(J: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Q^T J Q: the Jacobian of G = B - I on the admissible subspace spanned
    by Q, which B's Jacobian leaves invariant (its complement in the packed
    basis, absent from the paper's divergence-free basis, carries only the
    eigenvalue -1)."""
    return Q.T @ J @ Q


def admissible_restriction(J: np.ndarray, tol: float = 1e-9):
    """(Q^T J Q, Q) with Q from the range of J + I, for J the Jacobian of
    G = B - I of one step or of several (all share the admissible range; for
    many strongly damping steps pass a basis from one step to `restrict`
    instead, as the range of J + I then loses rank numerically)."""
    Q = admissible_basis(J + np.eye(J.shape[0]), tol)
    return restrict(J, Q), Q


def beaume_scale(lam: np.ndarray, T: float) -> np.ndarray:
    """lambda -> (1 + T)/T lambda for eigenvalues of G^Stokes_T."""
    return (1.0 + T) / T * np.asarray(lam)


def radius_containing(lam: np.ndarray, fraction: float = 0.95, center: complex = -1.0) -> float:
    """Smallest radius of a disc around `center` holding `fraction` of the
    eigenvalues."""
    d = np.sort(np.abs(np.asarray(lam) - center))
    k = int(np.ceil(fraction * d.size)) - 1
    return float(d[max(k, 0)])


def fraction_in_band(lam: np.ndarray, half_width: float = 0.2, center: float = -1.0) -> float:
    """Fraction of eigenvalues with |Re(lambda) - center| <= half_width."""
    lam = np.asarray(lam)
    return float(np.mean(np.abs(lam.real - center) <= half_width))


def summary(lam: np.ndarray) -> dict:
    lam = np.asarray(lam)
    return {"n": int(lam.size), "re_min": float(lam.real.min()), "re_max": float(lam.real.max()),
            "im_max": float(np.abs(lam.imag).max()),
            "radius95_about_-1": radius_containing(lam, 0.95),
            "fraction_re_within_0.2_of_-1": fraction_in_band(lam, 0.2)}
