"""The spectra tool on the GPU (Sec. 5): the dense Jacobian assembled from the
library's Jacobian actions equals the oracle's, J_Phi has rank at most the
dimension of the admissible subspace (so G_U has the eigenvalue -1 on the
rest), and about U = 0 the BEFE step's eigenvalues give back the analytic
Stokes eigenvalues."""
import math

import numpy as np
import pytest

from gpu_util import BOX, rel, say, to_dev
from oracle import pack as opack
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import SP_OP_PHI, SP_OP_RESIDUAL, spectra, synth

pytestmark = pytest.mark.gpu


def test_dense_jacobian_matches_oracle_and_rank():
    from paper_1804_05087_amd import Plan
    dims, re, dt = (8, 9, 8), 400.0, 100.0
    say("spectra dense 8x9x8")
    g = Grid(*dims, *BOX)
    B = Befe(g, re, dt)
    P = Plan(*dims, *BOX, re, dt)
    u = synth.perturbation_field(*dims, *BOX, seed=0)
    J = spectra.jacobian_dense(P, to_dev(u))
    n = P.packed_n
    Jref = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        Jref[:, i] = opack.pack(B.jvp(u, opack.unpack(e, g), "residual"), g) * dt
    say("dense rel", rel(J, Jref))
    assert rel(J, Jref) < 1e-12
    # J_Phi = J_G + I maps into the admissible subspace (dimension 590 here)
    sv = np.linalg.svd(J + np.eye(n), compute_uv=False)
    rank = int(np.sum(sv > 1e-9 * sv[0]))
    say("rank of J_Phi", rank)
    assert rank <= 590
    lam = spectra.eigenvalues(J)
    assert np.sum(np.abs(lam + 1) < 1e-6) >= n - 590
    say(spectra.summary(lam))


def test_stokes_eigenvalues_at_rest():
    """About U = 0 the nonlinear term drops out of the Jacobian, so the
    nonzero eigenvalues sigma of J_Phi are 1/(1 - dt mu) with mu those of the
    discrete Stokes operator: mu = -((j pi / 2)^2 + k^2)/Re (j >= 1) for the
    (0,0) mode's u, w and for the velocity component normal to k of every
    other mode (a Dirichlet Helmholtz problem)."""
    from paper_1804_05087_amd import Plan
    dims, re, dt = (4, 33, 4), 400.0, 1.0
    say("stokes eigenvalues 4x33x4")
    P = Plan(*dims, *BOX, re, dt)
    zero = P.empty().zero_()
    J = spectra.jacobian_dense(P, zero, op=SP_OP_PHI)
    sig = spectra.eigenvalues(J)
    sig = sig[np.abs(sig) > 1e-12]
    mu = (1 - 1 / sig) / dt
    alpha, gamma = 2 * math.pi / BOX[0], 2 * math.pi / BOX[1]
    for k2 in (0.0, alpha ** 2, gamma ** 2, alpha ** 2 + gamma ** 2):
        for j in range(1, 6):
            m = -((j * math.pi / 2) ** 2 + k2) / re
            err = np.min(np.abs(mu - m)) / abs(m)
            say("k2", round(k2, 3), "j", j, m, err)
            assert err < 1e-9
