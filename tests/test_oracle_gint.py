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
