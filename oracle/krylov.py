"""GMRES and Newton (test infrastructure only).

Sec. 2, eqs. linear/biglin: Newton solves G_U u = G(U) and sets U <- U - u.
The linear system is solved matrix free in the Krylov space spanned by
G(U), G_U G(U), ... (eq. Kspace) with GMRES (Saad & Schultz), unrestarted
(Sec. 2, the discussion of eq. CPU). The paper leaves the orthogonalisation,
the initial guess and the tolerance open; the readings used here are x0 = 0,
modified Gram-Schmidt, Givens rotations, stop when the least-squares residual
falls to rtol * ||b|| or after kmax iterations.

Hookstep (Sec. 3.2: the codes constrain the Newton step to a trusted region
of validity of the linearisation, the hookstep of Viswanath 2007): the step
is Q y with y minimising the GMRES model ||beta e_1 - Hbar y|| subject to
||y|| <= delta, written through the SVD Hbar = W diag(s) Z^T as
y(mu) = Z diag(s p / (s^2 + mu)) with p = W^T beta e_1 and mu >= 0 the
smallest value that meets the constraint. The radius delta follows the
standard trust-region rule (Dennis & Schnabel, ch. 6) on the ratio rho of the
actual to the predicted decrease of ||r||^2 (packed Euclidean norm, the GMRES
norm): a candidate with rho < 0.01 is rejected and delta halved (at most the
step length); after acceptance delta is halved if rho < 0.25 and doubled (up
to delta_max) if rho > 0.75 and the step lay on the boundary. The paper gives
no constants; these are the readings.

Pins (tests/test_oracle_krylov.py): on small dense systems the GMRES iterate
equals the least-squares minimiser over the Krylov basis (numpy.linalg.lstsq),
the reported residual equals the true residual, n iterations solve an n x n
system; Newton converges quadratically on a scalar/vector polynomial system
with a known root. The constrained step equals lstsq inside the ball, lies
on the sphere with the Lagrange condition (Hbar^T Hbar + mu I) y = Hbar^T b
otherwise, and beats a brute-force scan of the sphere; the trust-region
Newton reaches the root of arctan(A x) from starts where the full Newton step
diverges, and equals the full-step Newton when the radius never binds.
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


def gmres_basis(matvec, b: np.ndarray, kmax: int, rtol: float):
    """GMRES as above, returning the model instead of the iterate.

    Returns (V, Hbar, beta, k, relres): V the k+1 orthonormal basis vectors
    (rows), Hbar the unrotated (k+1) x k Hessenberg matrix with
    matvec(V[:k].T) = V.T @ Hbar, beta = ||b||, relres the final relative
    least-squares residual."""
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    V = np.zeros((kmax + 1, n))
    H = np.zeros((kmax + 1, kmax))
    V[0] = b / beta
    k_done = 0
    relres = 1.0
    for k in range(kmax):
        w = matvec(V[k])
        for i in range(k + 1):                      # modified Gram-Schmidt
            H[i, k] = float(np.dot(V[i], w))
            w = w - H[i, k] * V[i]
        H[k + 1, k] = float(np.linalg.norm(w))
        k_done = k + 1
        rhs = np.zeros(k + 2)
        rhs[0] = beta
        y = np.linalg.lstsq(H[:k + 2, :k + 1], rhs, rcond=None)[0]
        relres = float(np.linalg.norm(rhs - H[:k + 2, :k + 1] @ y) / beta)
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        if relres <= rtol or H[k + 1, k] == 0.0:
            break
    return V[:k_done + 1], H[:k_done + 1, :k_done], beta, k_done, relres


def hook_step(Hbar: np.ndarray, beta: float, delta: float):
    """The constrained least-squares step: min ||beta e_1 - Hbar y|| over
    ||y|| <= delta. Returns (y, mu, model_residual_norm)."""
    W, s, Zt = np.linalg.svd(Hbar, full_matrices=False)
    p = beta * W[0, :]
    rhs = np.zeros(Hbar.shape[0])
    rhs[0] = beta

    def y_of(mu):
        return Zt.T @ (s * p / (s * s + mu))

    y = y_of(0.0)
    mu = 0.0
    if np.linalg.norm(y) > delta:
        lo, hi = 0.0, float(np.max(s) * np.linalg.norm(p) / delta)
        for _ in range(400):                        # ||y(mu)|| decreases in mu
            mid = 0.5 * (lo + hi)
            if mid in (lo, hi):
                break
            if np.linalg.norm(y_of(mid)) > delta:
                lo = mid
            else:
                hi = mid
        mu = hi
        y = y_of(mu)
    return y, mu, float(np.linalg.norm(rhs - Hbar @ y))


def newton_hook(residual, jvp, norm, U0: np.ndarray, tol: float, max_newton: int,
                kmax: int, rtol: float, delta_init: float = 0.0, delta_min: float = 1e-12,
                delta_max: float = 1e300, max_trials: int = 10):
    """Trust-region Newton-GMRES with the hookstep (see the module notes).

    delta_init <= 0 starts from the length of the first unconstrained step.
    Returns (U, report) with per-step radius, trials, mu, step length, rho."""
    U = U0.copy()
    rep = {"res_norm": [], "krylov": [], "gmres_relres": [], "converged": False,
           "actions": 0, "delta": [], "trials": [], "mu": [], "step_norm": [], "rho": []}
    delta = min(delta_init, delta_max)
    G = residual(U)
    rep["actions"] += 1
    for it in range(max_newton + 1):
        rn = norm(G)
        rep["res_norm"].append(rn)
        if rn < tol:
            rep["converged"] = True
            break
        if it == max_newton:
            break
        V, Hbar, beta, k, relres = gmres_basis(lambda v: jvp(U, v), G, kmax, rtol)
        rep["actions"] += k
        rep["krylov"].append(k)
        rep["gmres_relres"].append(relres)
        if delta <= 0:
            delta = min(float(np.linalg.norm(hook_step(Hbar, beta, np.inf)[0])), delta_max)
        accepted = False
        for trial in range(1, max_trials + 1):
            y, mu, model = hook_step(Hbar, beta, delta)
            ny = float(np.linalg.norm(y))
            Uc = U - V[:k].T @ y
            Gc = residual(Uc)
            rep["actions"] += 1
            pred = beta * beta - model * model
            act = beta * beta - float(np.dot(Gc, Gc))
            rho = act / pred if pred > 0 else -np.inf
            if not rho >= 0.01:
                delta = 0.5 * min(delta, ny)
                if delta < delta_min:
                    break
                continue
            accepted = True
            rep["delta"].append(delta)
            rep["trials"].append(trial)
            rep["mu"].append(mu)
            rep["step_norm"].append(ny)
            rep["rho"].append(rho)
            U, G = Uc, Gc
            if rho < 0.25:
                delta = 0.5 * ny
            elif rho > 0.75 and mu > 0:
                delta = min(2.0 * delta, delta_max)
            break
        if not accepted:
            rep["failed"] = "trust region collapsed" if delta < delta_min else "no acceptable step"
            rep["res_norm"].append(rn)
            break
    rep["newton_iters"] = len(rep["krylov"])
    return U, rep


def newton_hook_befe(befe, U0_canonical: np.ndarray, tol: float, max_newton: int,
                     kmax: int, rtol: float, **hook):
    """newton_hook for r(U) = (Phi_dt(U) - U)/dt = 0 (as newton_befe)."""
    from . import pack
    g = befe.g

    def residual(x):
        return pack.pack(befe.residual(pack.unpack(x, g)), g)

    def jvp(x, dx):
        return pack.pack(befe.jvp(pack.unpack(x, g), pack.unpack(dx, g), "residual"), g)

    def norm(rx):
        return befe.norm_l2(pack.unpack(rx, g))

    x, rep = newton_hook(residual, jvp, norm, pack.pack(U0_canonical, g), tol, max_newton,
                         kmax, rtol, **hook)
    return pack.unpack(x, g), rep
