"""Pins of the oracle's BEFE step with laminar advection in the implicit
operator (the remedy proposed in Sec. 3.6)."""
import math

import numpy as np
import numpy.polynomial.chebyshev as npc

from oracle import advect
from oracle.befe import Befe
from oracle.grid import Grid
from oracle.stokes import StokesSolver
from paper_1804_05087_amd import synth

BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)


def test_y_matrix_is_chebyshev_multiplication_by_y():
    rng = np.random.default_rng(0)
    for N in (4, 8, 16):
        a = rng.standard_normal(N + 1)
        ref = npc.chebmulx(a)          # N+2 coefficients
        assert np.allclose(advect.y_matrix(N) @ a, ref[:N + 1], atol=1e-15)


def test_laminar_advection_against_the_physical_grid():
    """(U_lam . grad) u + (u . grad) U_lam = y du/dx + v e_x evaluated at the
    collocation points (y_j = cos(pi j / N)) from Fourier derivatives, then
    analysed; equal to -M u in the coefficients 0..N-2 (the product y du/dx
    has degree N+1, whose top term aliases onto T_{N-1} only)."""
    dims = (8, 17, 8)
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, 1.0, modes=[(0, 0)])
    u = synth.random_spectral(*dims, seed=3)
    N = g.N
    y = np.cos(np.pi * np.arange(N + 1) / N)
    ikx = (1j * g.kx())[:, None, None]
    vals = np.einsum("jn,cikn->cikj", B.T, ikx[None] * u)   # du/dx at y_j
    v = np.einsum("jn,ikn->ikj", B.T, u[1])
    phys = y * vals
    phys[0] += v
    coef = np.einsum("nj,cikj->cikn", B.Tinv, phys)
    M = advect.laminar_advection(g, u)
    assert np.abs((coef + M)[..., :N - 1]).max() < 1e-13 * np.abs(M).max()


def test_laminar_flow_is_a_fixed_point():
    dims = (8, 9, 8)
    g = Grid(*dims, *BOX)
    A = advect.AdvBefe(g, 400.0, 100.0)
    lam = synth.laminar_field(*dims)
    assert np.abs(A.phi(lam) - lam).max() < 1e-14


def test_increment_identity():
    """Phi~(u) - u = S~_0[L u + N(u)]: the right-hand side evaluated without
    any solve on u (spectral Laplacian, nonlinear term), the solve with
    no-slip walls."""
    dims = (8, 9, 8)
    g = Grid(*dims, *BOX)
    for dt in (1.0, 100.0):
        A = advect.AdvBefe(g, 400.0, dt)
        u = synth.perturbation_field(*dims, *BOX, seed=5, energy=0.05)
        lhs = A.phi(u) - u
        rhs = A.solver.solve(A.laplacian(u) / A.re + A.nonlinear(u)) * 1.0
        # solve(g) solves (L + M - 1/dt) phi - grad p = -g; the increment d of
        # Phi~ solves it with g = L u + N(u) scaled by dt / dt: see the header
        assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(lhs)


def test_streamwise_independent_modes_decouple():
    dims = (8, 9, 8)
    g = Grid(*dims, *BOX)
    re, dt = 400.0, 10.0
    S = StokesSolver(g, re, dt)
    Sa = advect.AdvectedSolver(g, re, dt)
    rhs = synth.random_spectral(*dims, seed=7)
    a = Sa.solve(rhs)
    s = S.solve(rhs)
    for j in range(1, g.nzh - 1):            # m_x = 0, m_z != 0
        assert np.allclose(a[1:, 0, j], s[1:, 0, j], rtol=0, atol=1e-13)
        g2 = rhs.copy()
        g2[0, 0, j] = rhs[0, 0, j] - s[1, 0, j]
        assert np.allclose(a[0, 0, j], S.solve(g2)[0, 0, j], rtol=0, atol=1e-13)
    # m_x != 0: the advection changes the solution
    assert np.abs(a[:, 1, 1] - s[:, 1, 1]).max() > 1e-3 * np.abs(s[:, 1, 1]).max()
