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
