"""Pins for the oracle's implicit solve (I - dt L)^{-1} with constraints (CPU).

* Manufactured solutions: divergence-free, no-slip polynomial velocities of
  degree <= N-2 with an arbitrary polynomial pressure satisfy the tau system
  exactly, so the solver must return them; the right-hand side is formed by
  applying the operator with numpy's Chebyshev-series derivative (chebder),
  not with the oracle's derivative matrix.
* The (0,0) Dirichlet Helmholtz problem (1/Re)u'' - u/dt = -c has the closed
  form u = c dt (1 - cosh(beta y)/cosh(beta)), beta^2 = Re/dt.
* Eigenvalues of the homogeneous solve at U = 0 reproduce the analytic Stokes
  eigenvalues of the channel (paper Sec. 3.5 discusses these as the stiff
  outliers of L + N_U).
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C
from scipy.optimize import brentq

from oracle import cheb
from oracle.grid import Grid
from oracle.stokes import StokesSolver
from paper_1804_05087_amd import synth

BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)


def _pad(a, n1):
    out = np.zeros(n1, dtype=complex)
    out[: len(a)] = a
    return out


def _d(a, n1, order=1):
    re = C.chebder(np.real(a), order) if len(a) > order else np.zeros(1)
    im = C.chebder(np.imag(a), order) if len(a) > order else np.zeros(1)
    return _pad(re, n1) + 1j * _pad(im, n1)


def _mul(a, b, n1):
    """Product of complex Chebyshev series a (complex) and b (real)."""
    return _pad(C.chebmul(np.real(a), b), n1) + 1j * _pad(C.chebmul(np.imag(a), b), n1)


def _manufactured(N, kx, kz, re, inv_dt, rng):
    n1 = N + 1
    k = math.hypot(kx, kz)
    q2 = np.array([3 / 8, 0, -1 / 2, 0, 1 / 8])       # (1 - y^2)^2
    q1 = np.array([1 / 2, 0, -1 / 2])                  # 1 - y^2
    a = rng.standard_normal(N - 5) + 1j * rng.standard_normal(N - 5)   # deg N-6
    b = rng.standard_normal(N - 3) + 1j * rng.standard_normal(N - 3)   # deg N-4
    v = _mul(a, q2, n1)                     # deg <= N-2, v = Dv = 0 at walls
    upar = 1j * _d(v, n1) / k
    uperp = _mul(b, q1, n1)                 # deg <= N-2, zero at walls
    u = (kx * upar + kz * uperp) / k
    w = (kz * upar - kx * uperp) / k
    p = rng.standard_normal(n1) + 1j * rng.standard_normal(n1)
    k2 = kx * kx + kz * kz

    def op(f):
        return (_d(f, n1, 2) - k2 * f) / re - inv_dt * f

    gu = -(op(u) - 1j * kx * p)
    gv = -(op(v) - _d(p, n1))
    gw = -(op(w) - 1j * kz * p)
    return np.stack([u, v, w]), np.stack([gu, gv, gw])


@pytest.mark.parametrize("dims,re,dt", [((8, 17, 8), 400.0, 100.0),
                                        ((16, 33, 16), 1000.0, 1.0),
                                        ((8, 25, 8), 400.0, 1e-3),
                                        ((8, 17, 8), 400.0, np.inf)])
def test_manufactured_solutions(dims, re, dt):
    nx, ny, nz = dims
    g = Grid(nx, ny, nz, *BOX)
    modes = [(1, 0), (nx - 1, 0), (0, 1), (2, 3), (nx - 2, 2), (nx // 2 - 1, nz // 2 - 1)]
    S = StokesSolver(g, re, dt, modes=modes)
    rng = np.random.default_rng(11)
    kx, kz = g.kx(), g.kz()
    gf = g.zeros()
    ref = g.zeros()
    for (i, j) in modes:
        uvw, gg = _manufactured(g.N, kx[i], kz[j], re, S.inv_dt, rng)
        gf[:, i, j] = gg
        ref[:, i, j] = uvw
    got = S.solve(gf)
    for (i, j) in modes:
        err = np.abs(got[:, i, j] - ref[:, i, j]).max() / np.abs(ref[:, i, j]).max()
        assert err < 1e-12, (i, j, err)


@pytest.mark.parametrize("re,dt", [(400.0, 100.0), (400.0, 1.0), (1000.0, 10.0)])
def test_mean_mode_closed_form(re, dt):
    g = Grid(4, 41, 4, *BOX)
    S = StokesSolver(g, re, dt, modes=[(0, 0)])
    c = 0.37
    gf = g.zeros()
    gf[0, 0, 0, 0] = c
    gf[2, 0, 0, 0] = -2 * c
    out = S.solve(gf)
    beta = math.sqrt(re / dt)
    y = cheb.points(g.N)
    vals = cheb.synthesis(g.N) @ out[0, 0, 0].real
    ref = c * dt * (1 - np.cosh(beta * y) / np.cosh(beta))
    assert np.abs(vals - ref).max() < 1e-12 * max(1, np.abs(ref).max())
    valsw = cheb.synthesis(g.N) @ out[2, 0, 0].real
    assert np.abs(valsw + 2 * ref).max() < 2e-12 * max(1, np.abs(ref).max())
    assert np.abs(out[1, 0, 0]).max() == 0.0


def test_mean_mode_wall_values():
    g = Grid(4, 17, 4, *BOX)
    S = StokesSolver(g, 400.0, 100.0, modes=[(0, 0)])
    out = S.solve(g.zeros(), 1.0, -1.0)
    # with g = 0 and walls +-1 the solution of u''/Re - u/dt = 0 is sinh(beta y)/sinh(beta)
    beta = math.sqrt(400.0 / 100.0)
    y = cheb.points(g.N)
    vals = cheb.synthesis(g.N) @ out[0, 0, 0].real
    assert np.abs(vals - np.sinh(beta * y) / np.sinh(beta)).max() < 1e-12


def _analytic_stokes(k, re, count):
    """Lowest channel Stokes eigenvalues mu for wavenumber k (k > 0)."""
    mus = []
    for j in range(1, count + 3):                       # Dirichlet family (u_perp)
        mus.append(-((j * math.pi / 2) ** 2 + k * k) / re)
    # v family: even s tan s = -k tanh k ; odd s cot s = k coth k
    fe = lambda s: s * math.sin(s) + k * math.tanh(k) * math.cos(s)
    fo = lambda s: s * math.cos(s) - k / math.tanh(k) * math.sin(s)
    for f in (fe, fo):
        xs = np.linspace(1e-6, (count + 4) * math.pi, 20000)
        vals = [f(x) for x in xs]
        for a, b, fa, fb in zip(xs[:-1], xs[1:], vals[:-1], vals[1:]):
            if fa * fb < 0:
                s = brentq(f, a, b, xtol=1e-15)
                if s > 1e-3:
                    mus.append(-(s * s + k * k) / re)
    return np.sort(np.array(mus))[::-1][:count]


@pytest.mark.parametrize("ny,tol", [(17, 5e-3), (33, 1e-10), (49, 1e-10)])
def test_stokes_eigenvalues(ny, tol):
    g = Grid(8, ny, 8, *BOX)
    re, dt = 400.0, 1.0
    modes = [(1, 0), (1, 1), (0, 2)]
    S = StokesSolver(g, re, dt, modes=modes + [(0, 0)])
    for (i, j) in modes:
        k = math.hypot(g.kx()[i], g.kz()[j])
        M = S.mode_operator(i, j) / dt
        sig = np.linalg.eigvals(M)
        sig = sig[np.abs(sig) > 1e-12]
        assert len(sig) == 2 * g.N - 4
        mu = (1 - 1 / sig) / dt
        mu = mu[np.argsort(-mu.real)]
        ref = _analytic_stokes(k, re, 11)
        got = np.sort(mu.real)[::-1][:11]
        assert np.abs(mu[:11].imag).max() < 1e-8
        assert np.abs(got - ref).max() / np.abs(ref).max() < tol, (i, j, got, ref)
    # (0,0): Dirichlet family for u and for w
    sig = np.linalg.eigvals(S.mean_operator() / dt)
    sig = sig[np.abs(sig) > 1e-12]
    mu = np.sort(((1 - 1 / sig) / dt).real)[::-1][:5]
    ref = np.array([-((j * math.pi / 2) ** 2) / re for j in range(1, 6)])
    assert np.abs(mu - ref).max() / np.abs(ref).max() < tol


def test_solutions_are_divergence_free_and_no_slip():
    g = Grid(8, 17, 8, *BOX)
    S = StokesSolver(g, 400.0, 10.0)
    rhs = synth.random_spectral(8, 17, 8, seed=5)
    out = S.solve(rhs, 1.0, -1.0)
    D = cheb.derivative(g.N)
    div = 1j * g.kx()[:, None, None] * out[0] + cheb.apply_y(D, out[1]) + \
        1j * g.kz()[None, :, None] * out[2]
    assert np.abs(div).max() < 1e-13 * np.abs(out).max()
    top, bot = cheb.values_at_walls(g.N)
    t, b = out @ top, out @ bot
    t[0, 0, 0] -= 1.0
    b[0, 0, 0] += 1.0
    assert np.abs(t).max() < 1e-14 and np.abs(b).max() < 1e-14


def test_adjoint_solve_equals_conjugate_transpose_of_explicit_operator():
    """solve_adjoint (one solve with A^H per mode) against the definition of the
    adjoint: the conjugate transpose of the explicit map g -> phi assembled
    column by column from forward solves (mode_operator, mean_operator)."""
    import math
    g = Grid(6, 13, 8, 2 * math.pi / 1.14, 2 * math.pi / 2.5)
    S = StokesSolver(g, 400.0, 10.0)
    rng = np.random.default_rng(7)
    w = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    got = S.solve_adjoint(w)
    for (i, j) in S.modes:
        if (i, j) == (0, 0):
            M = S.mean_operator()
            for c in (0, 2):
                ref = M.T @ w[c, 0, 0].real
                assert np.abs(got[c, 0, 0] - ref).max() <= 1e-14 * np.abs(ref).max()
            assert not np.any(got[1, 0, 0])
            continue
        ref = (S.mode_operator(i, j).conj().T @ w[:, i, j, :].reshape(-1)).reshape(3, g.ny)
        assert np.abs(got[:, i, j] - ref).max() <= 1e-14 * np.abs(ref).max(), (i, j)
