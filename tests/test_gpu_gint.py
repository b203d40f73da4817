"""GPU parity of the multi-step time-integration operator (Sec. 2, eq. Gint):
r = (Phi_dt^n(U) - U)/(n dt), its chain-rule Jacobian action and the
trust-region Newton on it, against the oracle's plain composition."""
import math

import numpy as np
import pytest

from gpu_util import BOX, rel, say, to_dev, to_np
from oracle import gint
from oracle import pack as opack
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import SP_OP_PHI, SP_OP_RESIDUAL, SPError, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("dims,n,dt", [((8, 9, 8), 8, 0.125), ((16, 17, 16), 5, 0.2),
                                       ((12, 21, 24), 3, 0.5)])
def test_residual_and_jvp_parity(dims, n, dt):
    from paper_1804_05087_amd import Plan
    say("gint", dims, n, dt)
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, dt)
    P = Plan(*dims, *BOX, 400.0, dt)
    P.set_steps(n)
    u = synth.perturbation_field(*dims, *BOX, seed=1, energy=0.05)
    du = synth.random_admissible(*dims, *BOX, seed=2)
    r_ref = gint.residual(B, u, n)
    r = to_np(P.residual(to_dev(u)))
    say("residual", rel(r, r_ref))
    assert rel(r, r_ref) < TOL
    j_ref = gint.jvp(B, u, du, n)
    j = to_np(P.jvp(to_dev(u), to_dev(du), SP_OP_RESIDUAL))
    say("jvp", rel(j, j_ref))
    assert rel(j, j_ref) < TOL
    # the one-step action about the same point is unaffected by the chain
    jp = to_np(P.jvp_lin(to_dev(du), SP_OP_PHI))
    assert rel(jp, B.jvp(u, du, "phi")) < TOL
    with pytest.raises(SPError):
        P.vjp(to_dev(u), to_dev(du), SP_OP_RESIDUAL)
    P.set_steps(1)
    r1 = to_np(P.residual(to_dev(u)))
    assert rel(r1, B.residual(u)) < TOL


@pytest.mark.parametrize("scheme", [0, 1])
def test_newton_hookstep_on_gint_matches_oracle(scheme):
    from paper_1804_05087_amd import Plan
    dims, n, dt = (8, 9, 8), 4, 0.25
    say("gint newton", dims, n, dt, "scheme", scheme)
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, dt)
    P = Plan(*dims, *BOX, 400.0, dt)
    P.set_steps(n)
    P.set_scheme(scheme)
    u0 = synth.perturbation_field(*dims, *BOX, seed=0, energy=1e-2)
    _, ref = gint.newton_hook_gint(B, u0, n, 1e-10, 3, 15, 1e-6, sbdf2=bool(scheme))
    u = to_dev(u0)
    rep = P.newton_hookstep(u, max_newton=3, max_krylov=15, gmres_rtol=1e-6, newton_tol=1e-10)
    say("gpu", rep["res_norm"], rep["krylov"], rep["rho"])
    say("ref", ref["res_norm"], ref["krylov"], ref["rho"])
    assert rep["krylov"] == ref["krylov"]
    assert rep["trials"] == ref["trials"]
    for a, b in zip(rep["res_norm"], ref["res_norm"]):
        assert abs(a - b) <= 1e-8 * b
    for a, b in zip(rep["rho"], ref["rho"]):
        assert abs(a - b) <= 1e-6


@pytest.mark.parametrize("dims,n,tau", [((8, 9, 8), 6, 0.125), ((16, 17, 16), 4, 0.2),
                                        ((12, 21, 24), 3, 0.5)])
def test_sbdf2_residual_and_jvp_parity(dims, n, tau):
    """The SBDF2 integrator (scheme 1, implicit step tau = the plan's dt, time
    step 1.5 tau) against the oracle's SBDF2 map and chain rule."""
    from paper_1804_05087_amd import Plan
    say("sbdf2", dims, n, tau)
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, tau)
    P = Plan(*dims, *BOX, 400.0, tau)
    P.set_steps(n)
    P.set_scheme(1)
    u = synth.perturbation_field(*dims, *BOX, seed=1, energy=0.05)
    du = synth.random_admissible(*dims, *BOX, seed=2)
    r_ref = gint.sbdf2_residual(B, u, n)
    r = to_np(P.residual(to_dev(u)))
    say("residual", rel(r, r_ref))
    assert rel(r, r_ref) < TOL
    j_ref = gint.sbdf2_jvp(B, u, du, n)
    j = to_np(P.jvp(to_dev(u), to_dev(du), SP_OP_RESIDUAL))
    say("jvp", rel(j, j_ref))
    assert rel(j, j_ref) < TOL
    # a second action about the same base reuses the trajectory
    j2 = to_np(P.jvp_lin(to_dev(du), SP_OP_RESIDUAL))
    assert rel(j2, j_ref) < TOL
    # one step of SBDF2 is a BEFE step of tau, residual scaled by 1 / 1.5
    P.set_steps(1)
    assert rel(to_np(P.residual(to_dev(u))), B.residual(u) / 1.5) < TOL
    P.set_scheme(0)
    assert rel(to_np(P.residual(to_dev(u))), B.residual(u)) < TOL


def test_sbdf2_rejects_mixed_precision_and_bad_values():
    from paper_1804_05087_amd import SP_MIXED, Plan
    dims = (8, 9, 8)
    P = Plan(*dims, *BOX, 400.0, 0.125)
    P.set_steps(4)
    with pytest.raises(SPError):
        P.set_scheme(2)
    P.set_scheme(1)
    P.set_precision(SP_MIXED)
    u = to_dev(synth.perturbation_field(*dims, *BOX, seed=1))
    with pytest.raises(SPError):
        P.residual(u)
    with pytest.raises(SPError):
        P.linearize(u)
