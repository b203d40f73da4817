"""The spectra tool on the GPU (Sec. 3.5): the dense Jacobian assembled from the
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


@pytest.mark.parametrize("op", [SP_OP_PHI, SP_OP_RESIDUAL])
def test_jacobian_columns_equal_single_actions(op):
    """sp_jacobian_columns forms each column on the device from the same
    kernels as unpack + sp_jvp_lin + pack, so a sub-range of columns equals
    the one-at-a-time route bit for bit."""
    import torch
    from paper_1804_05087_amd import Plan
    dims, re, dt = (12, 17, 12), 500.0, 1.0
    say("jacobian columns 12x17x12 op", op)
    P = Plan(*dims, *BOX, re, dt)
    u = to_dev(synth.perturbation_field(*dims, *BOX, seed=2, energy=1e-2))
    P.linearize(u)
    n = P.packed_n
    first, count = n // 3, 37
    cols = P.jacobian_columns(op, first, count).cpu().numpy()
    e = torch.zeros(n, dtype=torch.float64, device=P.device)
    for c in range(count):
        e.zero_()
        e[first + c] = 1.0
        ref = P.pack(P.jvp_lin(P.unpack(e), op)).cpu().numpy()
        assert np.array_equal(cols[c], ref), c
    # the last column of the basis and an empty range
    last = P.jacobian_columns(op, n - 1, 1).cpu().numpy()
    e.zero_()
    e[n - 1] = 1.0
    assert np.array_equal(last[0], P.pack(P.jvp_lin(P.unpack(e), op)).cpu().numpy())
    assert P.jacobian_columns(op, n, 0).shape == (0, n)


def test_jacobian_columns_rejects_bad_ranges():
    import ctypes as C
    import torch
    from paper_1804_05087_amd import Plan, SPError
    dims = (8, 9, 8)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    n = P.packed_n
    buf = torch.zeros((2, n), dtype=torch.float64, device=P.device)
    with pytest.raises(SPError):  # no base state yet
        P.jacobian_columns(SP_OP_PHI, 0, 2, out=buf)
    P.linearize(to_dev(synth.perturbation_field(*dims, *BOX, seed=0)))
    for first, count, ld in ((-1, 1, n), (n - 1, 2, n), (0, 1, n - 1)):
        st = P.lib.sp_jacobian_columns(P.h, SP_OP_PHI, first, count, C.c_void_p(buf.data_ptr()), ld)
        assert st != 0, (first, count, ld)
    st = P.lib.sp_jacobian_columns(P.h, 7, 0, 1, C.c_void_p(buf.data_ptr()), n)
    assert st != 0
    assert torch.count_nonzero(buf).item() == 0


@pytest.mark.parametrize("scheme", [0, 1])
def test_jacobian_columns_of_the_multistep_operator_match_oracle(scheme):
    """Dense-Jacobian columns of the time-integration operator (BEFE or SBDF2
    steps, 3 of them) against the oracle's chain rule on the same unit
    vectors, a sample of 24 columns spread over the packed basis."""
    from oracle import gint
    from paper_1804_05087_amd import Plan
    dims, re, dt, n = (8, 9, 8), 400.0, 0.2, 3
    say("multistep jacobian columns, scheme", scheme)
    g = Grid(*dims, *BOX)
    B = Befe(g, re, dt)
    P = Plan(*dims, *BOX, re, dt)
    P.set_steps(n)
    P.set_scheme(scheme)
    u = synth.perturbation_field(*dims, *BOX, seed=4, energy=0.05)
    P.linearize(to_dev(u))
    m = P.packed_n
    jv = gint.sbdf2_jvp if scheme else gint.jvp
    for first in np.linspace(0, m - 1, 24).astype(int):
        col = P.jacobian_columns(SP_OP_RESIDUAL, int(first), 1).cpu().numpy()[0]
        e = np.zeros(m)
        e[first] = 1.0
        ref = opack.pack(jv(B, u, opack.unpack(e, g), n), g)
        assert rel(col, ref) < 1e-12, (first, rel(col, ref))
