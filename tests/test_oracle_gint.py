"""Pins of the oracle's multi-step time-integration operator (Sec. 2, eq. Gint)."""
import math

import numpy as np

from oracle import gint
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)
DIMS = (8, 9, 8)


def test_laminar_flow_is_a_root():
    g = Grid(*DIMS, *BOX)
    B = Befe(g, 400.0, 0.125)
    lam = synth.laminar_field(*DIMS)
    r = gint.residual(B, lam, 8)
    assert np.abs(r).max() < 1e-14


def test_one_step_is_the_stokes_residual():
    g = Grid(*DIMS, *BOX)
    B = Befe(g, 400.0, 2.0)
    u = synth.perturbation_field(*DIMS, *BOX, seed=3)
    assert np.array_equal(gint.residual(B, u, 1), B.residual(u))


def test_jvp_matches_central_differences_to_second_order():
    g = Grid(*DIMS, *BOX)
    B = Befe(g, 400.0, 0.25)
    u = synth.perturbation_field(*DIMS, *BOX, seed=4, energy=0.05)
    du = synth.random_admissible(*DIMS, *BOX, seed=5)
    n = 4
    J = gint.jvp(B, u, du, n)
    errs = []
    for h in (1e-3, 5e-4):
        fd = (gint.residual(B, u + h * du, n) - gint.residual(B, u - h * du, n)) / (2 * h)
        errs.append(np.linalg.norm(fd - J) / np.linalg.norm(J))
    # a quartic-and-higher composition: central differences err at O(h^2)
    assert errs[0] < 1e-5
    assert 3.0 < errs[0] / errs[1] < 5.0
    # the chain taken at the wrong points (all at U_0) is visibly different
    v = du
    for _ in range(n):
        v = B.jvp(u, v, "phi")
    wrong = (v - du) / (n * B.dt)
    assert np.linalg.norm(wrong - J) > 1e3 * errs[0] * np.linalg.norm(J)


def test_bef_euler_is_first_order_in_time():
    g = Grid(*DIMS, *BOX)
    u = synth.perturbation_field(*DIMS, *BOX, seed=6, energy=0.05)
    T = 1.0
    finals = {}
    for n in (8, 16, 32):
        B = Befe(g, 400.0, T / n)
        finals[n] = gint.trajectory(B, u, n)[-1]
    d1 = np.linalg.norm(finals[8] - finals[16])
    d2 = np.linalg.norm(finals[16] - finals[32])
    assert 1.8 < d1 / d2 < 2.2


# ---- SBDF2 as the integrator -------------------------------------------------------------

def test_sbdf2_laminar_flow_is_a_root():
    g = Grid(*DIMS, *BOX)
    B = Befe(g, 400.0, 2.0 / 3.0 * 0.125)
    lam = synth.laminar_field(*DIMS)
    assert np.abs(gint.sbdf2_residual(B, lam, 8)).max() < 1e-13


def test_sbdf2_first_step_is_a_befe_step_of_tau():
    # with u_{-1} = u_0 the first step reads (I - tau L) u_1 = u_0 + tau N(u_0)
    g = Grid(*DIMS, *BOX)
    B = Befe(g, 400.0, 0.5)
    u = synth.perturbation_field(*DIMS, *BOX, seed=3)
    r1 = gint.sbdf2_residual(B, u, 1)
    ref = B.residual(u) / 1.5
    assert np.linalg.norm(r1 - ref) <= 1e-13 * np.linalg.norm(ref)


def test_sbdf2_jvp_matches_central_differences_to_second_order():
    g = Grid(*DIMS, *BOX)
    B = Befe(g, 400.0, 0.25)
    u = synth.perturbation_field(*DIMS, *BOX, seed=4, energy=0.05)
    du = synth.random_admissible(*DIMS, *BOX, seed=5)
    n = 4
    J = gint.sbdf2_jvp(B, u, du, n)
    errs = []
    for h in (1e-3, 5e-4):
        fd = (gint.sbdf2_residual(B, u + h * du, n) - gint.sbdf2_residual(B, u - h * du, n)) / (2 * h)
        errs.append(np.linalg.norm(fd - J) / np.linalg.norm(J))
    assert errs[0] < 1e-5
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_sbdf2_about_rest_follows_the_bdf2_recurrence():
    """About U = 0 with walls at rest (a fixed point, so the whole trajectory
    stays at 0) the linearised product vanishes, so on an eigenvector v of
    one BEFE step of tau (eigenvalue mu) the n SBDF2 steps act as the scalar
    recurrence d_{k+1} = mu (4 d_k - d_{k-1}) / 3 with d_{-1} = d_0 = 1: the
    weights 4/3 and -1/3 of the scheme and its start are fixed by this."""
    from oracle import pack as opack
    dims = (4, 9, 4)
    g = Grid(*dims, *BOX)
    tau = 0.3
    B = Befe(g, 50.0, tau, wall_upper=0.0, wall_lower=0.0)  # U = 0 is then a fixed point
    zero = np.zeros((3, dims[0], dims[2] // 2 + 1, dims[1]), dtype=np.complex128)
    m = len(opack.pack(zero, g))
    Jphi = np.empty((m, m))
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        Jphi[:, i] = opack.pack(B.jvp(zero, opack.unpack(e, g), "phi"), g)
    # the step maps into its range (the admissible fields) and annihilates a
    # large complement; eigenpairs are taken on the range, Q^T J Q with Q an
    # orthonormal basis of it, and lifted back (J Q y = Q (Q^T J Q) y there)
    U, sv, _ = np.linalg.svd(Jphi)
    Q = U[:, sv > 1e-9 * sv[0]]
    mu, Y = np.linalg.eig(Q.T @ Jphi @ Q)
    n = 5
    checked = 0
    for k in np.argsort(-np.abs(mu)):
        if abs(mu[k].imag) > 1e-12 or not 0.05 < mu[k].real < 0.98:
            continue
        v = Q @ Y[:, k].real
        assert np.linalg.norm(Jphi @ v - mu[k].real * v) <= 1e-10 * np.linalg.norm(v)
        d_prev, d = 1.0, 1.0
        for _ in range(n):
            d_prev, d = d, mu[k].real * (4.0 * d - d_prev) / 3.0
        Jv = opack.pack(gint.sbdf2_jvp(B, zero, opack.unpack(v, g), n), g) * (1.5 * n * tau) + v
        assert np.linalg.norm(Jv - d * v) <= 1e-10 * np.linalg.norm(v), (mu[k], d)
        checked += 1
        if checked == 6:
            break
    assert checked >= 3
