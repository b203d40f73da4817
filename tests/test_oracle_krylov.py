"""Pins for the oracle's GMRES and Newton (CPU).

GMRES (Sec. 2, eq. Kspace) minimises ||b - A x|| over the Krylov space
span{b, Ab, ..., A^{k-1} b}; the pin is numpy.linalg.lstsq over an explicitly
built Krylov basis. Newton (Sec. 2, eqs. linear, biglin) must converge
quadratically to a known root of a polynomial system.
"""
import numpy as np

from oracle import krylov


def test_gmres_equals_krylov_least_squares():
    rng = np.random.default_rng(0)
    n = 30
    A = np.eye(n) * 3 + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    for k in (1, 3, 7, 15):
        x, hist, kd = krylov.gmres(lambda v: A @ v, b, k, 0.0)
        assert kd == k
        K = np.zeros((n, k))
        v = b.copy()
        for i in range(k):
            K[:, i] = v / np.linalg.norm(v)
            v = A @ v
        c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
        xref = K @ c
        assert np.linalg.norm(x - xref) < 1e-8 * np.linalg.norm(xref)
        true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        ref_res = np.linalg.norm(b - A @ xref) / np.linalg.norm(b)
        assert abs(true - hist[-1]) < 1e-12
        assert true <= ref_res * (1 + 1e-10)


def test_gmres_full_dimension_solves():
    rng = np.random.default_rng(1)
    n = 12
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal(n)
    x, hist, k = krylov.gmres(lambda v: A @ v, b, n, 1e-14)
    assert np.linalg.norm(A @ x - b) < 1e-12 * np.linalg.norm(b)


def test_newton_quadratic_convergence():
    # G(U) = U^2 - c (componentwise) + small coupling, root known by construction
    rng = np.random.default_rng(2)
    n = 8
    root = 1.0 + rng.random(n)
    M = 0.1 * rng.standard_normal((n, n))

    def G(U):
        return U * U + M @ U - (root * root + M @ root)

    def JG(U, du):
        return 2 * U * du + M @ du

    U, rep = krylov.newton(G, JG, np.linalg.norm, root + 0.05, 1e-13, 10, n, 1e-14)
    assert rep["converged"]
    assert np.abs(U - root).max() < 1e-12
    r = rep["res_norm"]
    # quadratic: log error roughly doubles once in the asymptotic regime
    assert r[2] < 10 * r[1] ** 2 / r[0] ** 0 + 1e-14


# ---------------------------------------------------------------- hookstep
# The constrained step min ||b - Hbar y|| over ||y|| <= delta (Sec. 3.2, the
# hookstep of Viswanath 2007) is pinned by what fixes it mathematically: the
# unconstrained least-squares solution when it fits, otherwise a point of the
# sphere ||y|| = delta satisfying the Lagrange condition with mu > 0, and no
# point of the ball doing better.

def _hessenberg(k, seed):
    """A well-conditioned (k+1) x k upper Hessenberg matrix: Arnoldi of a
    shifted random matrix."""
    rng = np.random.default_rng(seed)
    n = 2 * k + 3
    A = 3 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    V, H, beta, kd, _ = krylov.gmres_basis(lambda v: A @ v, b, k, 0.0)
    assert kd == k
    assert np.allclose(A @ V[:k].T, V.T @ H, atol=1e-12)
    return H, beta


def test_hook_step_inside_ball_is_least_squares():
    H, beta = _hessenberg(12, 3)
    rhs = np.zeros(13)
    rhs[0] = beta
    yls = np.linalg.lstsq(H, rhs, rcond=None)[0]
    y, mu, model = krylov.hook_step(H, beta, 1.5 * np.linalg.norm(yls))
    assert mu == 0.0
    assert np.linalg.norm(y - yls) < 1e-12 * np.linalg.norm(yls)
    assert abs(model - np.linalg.norm(rhs - H @ yls)) < 1e-13 * beta


def test_hook_step_on_sphere_satisfies_lagrange_condition():
    H, beta = _hessenberg(12, 4)
    rhs = np.zeros(13)
    rhs[0] = beta
    yls = np.linalg.lstsq(H, rhs, rcond=None)[0]
    for f in (0.9, 0.5, 0.1, 1e-3):
        delta = f * np.linalg.norm(yls)
        y, mu, model = krylov.hook_step(H, beta, delta)
        assert mu > 0
        assert abs(np.linalg.norm(y) - delta) < 1e-12 * delta
        lhs = (H.T @ H + mu * np.eye(12)) @ y
        assert np.linalg.norm(lhs - H.T @ rhs) < 1e-10 * np.linalg.norm(H.T @ rhs)
        assert abs(model - np.linalg.norm(rhs - H @ y)) < 1e-13 * beta


def test_hook_step_beats_a_scan_of_the_ball():
    # k = 2: the sphere is a circle, scanned densely; points inside the ball
    # are never better than the constrained minimiser
    H, beta = _hessenberg(2, 5)
    rhs = np.array([beta, 0.0, 0.0])
    yls = np.linalg.lstsq(H, rhs, rcond=None)[0]
    delta = 0.4 * np.linalg.norm(yls)
    y, mu, model = krylov.hook_step(H, beta, delta)
    th = np.linspace(0, 2 * np.pi, 200001)
    pts = delta * np.stack([np.cos(th), np.sin(th)])
    vals = np.linalg.norm(rhs[:, None] - H @ pts, axis=0)
    assert model <= vals.min() + 1e-12
    assert model >= vals.min() - 1e-6 * beta   # the scan finds the same minimum
    rng = np.random.default_rng(6)
    inside = rng.standard_normal((2, 5000))
    inside *= delta * rng.random(5000) ** 0.5 / np.linalg.norm(inside, axis=0)
    assert model <= np.linalg.norm(rhs[:, None] - H @ inside, axis=0).min() + 1e-12


def test_trust_region_newton_converges_where_full_newton_diverges():
    # G(x) = arctan(A x) has the single root x = 0; from ||A x0|| well above
    # ~1.39 the full Newton step overshoots and the iterates grow without bound
    rng = np.random.default_rng(7)
    n = 4
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag([1.0, 1.5, 2.0, 3.0]) @ Q.T
    x0 = Q @ np.array([2.0, -1.5, 1.0, 2.5])

    def G(x):
        return np.arctan(A @ x)

    def JG(x, dx):
        return (A @ dx) / (1.0 + (A @ x) ** 2)

    _, full = krylov.newton(G, JG, np.linalg.norm, x0, 1e-12, 6, n, 1e-14)
    assert not full["converged"]
    assert full["res_norm"][-1] > full["res_norm"][0]
    x, rep = krylov.newton_hook(G, JG, np.linalg.norm, x0, 1e-12, 40, n, 1e-14)
    assert rep["converged"], rep
    assert np.linalg.norm(x) < 1e-11
    assert max(rep["trials"]) > 1 or min(rep["rho"]) < 0.25   # the radius did bind
    assert all(r >= 0.01 for r in rep["rho"])


def test_trust_region_newton_equals_newton_when_unconstrained():
    rng = np.random.default_rng(8)
    n = 8
    root = 1.0 + rng.random(n)
    M = 0.1 * rng.standard_normal((n, n))

    def G(U):
        return U * U + M @ U - (root * root + M @ root)

    def JG(U, du):
        return 2 * U * du + M @ du

    U1, r1 = krylov.newton(G, JG, np.linalg.norm, root + 0.05, 1e-13, 10, n, 1e-14)
    U2, r2 = krylov.newton_hook(G, JG, np.linalg.norm, root + 0.05, 1e-13, 10, n, 1e-14,
                                delta_init=1e6)
    assert r2["converged"] and r1["converged"]
    assert all(m == 0.0 for m in r2["mu"]) and all(t == 1 for t in r2["trials"])
    assert len(r1["res_norm"]) == len(r2["res_norm"])
    for a, b in zip(r1["res_norm"], r2["res_norm"]):
        assert abs(a - b) <= 1e-10 * max(b, 1e-13)
