"""GMRES and Newton (test infrastructure only).

Sec. 2, eqs. linear/biglin: Newton solves G_U u = G(U) and sets U <- U - u.
The linear system is solved matrix free in the Krylov space spanned by
G(U), G_U G(U), ... (eq. Kspace) with GMRES (Saad & Schultz), unrestarted
(Sec. 2, the discussion of eq. CPU). The paper leaves the orthogonalisation,
the initial guess and the tolerance open; the readings used here are x0 = 0,
modified Gram-Schmidt, Givens rotations, stop when the least-squares residual
falls to rtol * ||b|| or after kmax iterations.

Pins (tests/test_oracle_krylov.py): on small dense systems the GMRES iterate
equals the least-squares minimiser over the Krylov basis (numpy.linalg.lstsq),
the reported residual equals the true residual, n iterations solve an n x n
system; Newton converges quadratically on a scalar/vector polynomial system
with a known root.
"""
from __future__ import annotations

import time

import numpy as np


def gmres(matvec, b: np.ndarray, kmax: int, rtol: float):
    """Unrestarted GMRES from x0 = 0. Returns (x, relres_history, k)."""
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    hist = []
    if beta == 0.0:
        return np.zeros_like(b), hist, 0
    V = np.zeros((kmax + 1, n))
    H = np.zeros((kmax + 1, kmax))
    cs = np.zeros(kmax)
    sn = np.zeros(kmax)
    gvec = np.zeros(kmax + 1)
    gvec[0] = beta
    V[0] = b / beta
    k_done = 0
    for k in range(kmax):
        w = matvec(V[k])
        for i in range(k + 1):                      # modified Gram-Schmidt
            H[i, k] = float(np.dot(V[i], w))
            w = w - H[i, k] * V[i]
        H[k + 1, k] = float(np.linalg.norm(w))
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        for i in range(k):                          # apply previous rotations
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        d = np.hypot(H[k, k], H[k + 1, k])
        cs[k] = H[k, k] / d
        sn[k] = H[k + 1, k] / d
        H[k, k] = d
        H[k + 1, k] = 0.0
        gvec[k + 1] = -sn[k] * gvec[k]
        gvec[k] = cs[k] * gvec[k]
        k_done = k + 1
        hist.append(abs(gvec[k + 1]) / beta)
        if abs(gvec[k + 1]) <= rtol * beta or H[k, k] == 0.0:
            break
    y = np.zeros(k_done)
    for i in range(k_done - 1, -1, -1):
        y[i] = (gvec[i] - np.dot(H[i, i + 1:k_done], y[i + 1:k_done])) / H[i, i]
    x = V[:k_done].T @ y
    return x, hist, k_done


def newton(residual, jvp, norm, U0: np.ndarray, tol: float, max_newton: int,
           kmax: int, rtol: float):
    """Newton-GMRES on packed vectors.

    residual(U) -> G(U); jvp(U, du) -> G_U du; norm(G) -> the stopping norm.
    Returns (U, report dict).
    """
    U = U0.copy()
    rep = {"res_norm": [], "krylov": [], "gmres_relres": [], "converged": False,
           "actions": 0}
    t0 = time.perf_counter()
    for it in range(max_newton + 1):
        G = residual(U)
        rep["actions"] += 1
        rn = norm(G)
        rep["res_norm"].append(rn)
        if rn < tol:
            rep["converged"] = True
            break
        if it == max_newton:
            break
        du, hist, k = gmres(lambda v: jvp(U, v), G, kmax, rtol)
        rep["actions"] += k
        rep["krylov"].append(k)
        rep["gmres_relres"].append(hist[-1] if hist else 0.0)
        U = U - du
    rep["seconds"] = time.perf_counter() - t0
    rep["newton_iters"] = len(rep["krylov"])
    return U, rep


def newton_befe(befe, U0_canonical: np.ndarray, tol: float, max_newton: int,
                kmax: int, rtol: float):
    """Newton-GMRES for r(U) = (Phi_dt(U) - U)/dt = 0 on packed vectors.

    The stopping norm is the volume-normalised L2 norm of r; GMRES works in
    the packed Euclidean inner product with the exact Jacobian J_r.
    Returns (U_canonical, report).
    """
    from . import pack
    g = befe.g

    def residual(x):
        return pack.pack(befe.residual(pack.unpack(x, g)), g)

    def jvp(x, dx):
        return pack.pack(befe.jvp(pack.unpack(x, g), pack.unpack(dx, g), "residual"), g)

    def norm(rx):
        return befe.norm_l2(pack.unpack(rx, g))

    x, rep = newton(residual, jvp, norm, pack.pack(U0_canonical, g), tol, max_newton,
                    kmax, rtol)
    return pack.unpack(x, g), rep
