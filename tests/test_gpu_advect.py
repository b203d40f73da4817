"""GPU parity of the BEFE step with the laminar advection in the implicit
operator (Sec. 3.6's proposed remedy) against the oracle's dense per-mode
solves: Phi~, its Jacobian action, the multi-step operator built on it, and
the aliasing and error contracts."""
import math

import numpy as np
import pytest

from gpu_util import BOX, rel, say, to_dev, to_np
from oracle import advect
from oracle.grid import Grid
from paper_1804_05087_amd import SP_OP_PHI, SP_OP_RESIDUAL, SPError, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("case", [((8, 9, 8), 400.0, 100.0), ((16, 17, 16), 400.0, 10.0),
                                  ((12, 21, 24), 1000.0, 1.0)])
def test_advected_step_and_jvp_parity(case):
    from paper_1804_05087_amd import Plan
    dims, re, dt = case
    say("advected", dims, re, dt)
    g = Grid(*dims, *BOX)
    A = advect.AdvBefe(g, re, dt)
    P = Plan(*dims, *BOX, re, dt)
    P.set_advection(True)
    u = synth.perturbation_field(*dims, *BOX, seed=2, energy=0.05)
    du = synth.random_admissible(*dims, *BOX, seed=3)
    ref = A.phi(u)
    got = to_np(P.befe_step(to_dev(u)))
    say("phi", rel(got, ref))
    assert rel(got, ref) < TOL
    r = to_np(P.residual(to_dev(u)))
    assert rel(r, A.residual(u)) < TOL
    j = to_np(P.jvp(to_dev(u), to_dev(du), SP_OP_RESIDUAL))
    jref = A.jvp(u, du, "residual")
    say("jvp", rel(j, jref))
    assert rel(j, jref) < TOL
    # out may alias u
    x = to_dev(u)
    P.befe_step(x, x)
    assert rel(to_np(x), ref) < TOL
    with pytest.raises(SPError):
        P.vjp(to_dev(u), to_dev(du), SP_OP_PHI)
    # switching back restores the Stokes step
    P.set_advection(False)
    from oracle.befe import Befe
    assert rel(to_np(P.befe_step(to_dev(u))), Befe(g, re, dt).phi(u)) < TOL


def test_advected_multistep_and_newton():
    """The time-integration operator composed of advected steps, and a
    hookstep Newton solve with the advected Jacobian reaching the laminar
    root from a small perturbation."""
    from oracle import gint
    from paper_1804_05087_amd import Plan
    dims, re, dt, n = (8, 9, 8), 400.0, 0.25, 4
    say("advected multistep")
    g = Grid(*dims, *BOX)
    A = advect.AdvBefe(g, re, dt)
    P = Plan(*dims, *BOX, re, dt)
    P.set_advection(True)
    P.set_steps(n)
    u = synth.perturbation_field(*dims, *BOX, seed=4, energy=0.05)
    du = synth.random_admissible(*dims, *BOX, seed=5)
    assert rel(to_np(P.residual(to_dev(u))), gint.residual(A, u, n)) < TOL
    assert rel(to_np(P.jvp(to_dev(u), to_dev(du), SP_OP_RESIDUAL)), gint.jvp(A, u, du, n)) < TOL
    P2 = Plan(*dims, *BOX, re, 100.0)
    P2.set_advection(True)
    x = to_dev(synth.perturbation_field(*dims, *BOX, seed=0, energy=1e-6))
    rep = P2.newton_hookstep(x, max_newton=6, max_krylov=60, gmres_rtol=1e-8, newton_tol=1e-12)
    say(rep["res_norm"], rep["krylov"])
    assert rep["converged"]
    lam = synth.laminar_field(*dims)
    assert np.abs(to_np(x) - lam).max() < 1e-9


def test_advected_mixed_precision():
    """FP32 transforms and contractions with the FP64 advected solve, against
    the FP64 oracle (same bound as the Stokes step's mixed path)."""
    from paper_1804_05087_amd import SP_MIXED, Plan
    dims, re, dt = (16, 17, 16), 400.0, 100.0
    say("advected mixed", dims)
    g = Grid(*dims, *BOX)
    A = advect.AdvBefe(g, re, dt)
    P = Plan(*dims, *BOX, re, dt, precision=SP_MIXED)
    P.set_advection(True)
    u = synth.perturbation_field(*dims, *BOX, seed=0)
    du = synth.random_admissible(*dims, *BOX, seed=1)
    e_phi = rel(to_np(P.befe_step(to_dev(u))), A.phi(u))
    e_jvp = rel(to_np(P.jvp(to_dev(u), to_dev(du), SP_OP_PHI)), A.jvp(u, du))
    say("mixed advected errors phi", e_phi, "jvp", e_jvp)
    assert e_phi < 2e-5 and e_jvp < 2e-5
    assert e_phi > 1e-12  # the FP32 path really ran


def test_invalid_arguments_are_rejected():
    from paper_1804_05087_amd import Plan
    P = Plan(8, 9, 8, *BOX, 400.0, 1.0)
    for bad in (0, -3, 100001):
        with pytest.raises(SPError):
            P.set_steps(bad)
    u = to_dev(synth.perturbation_field(8, 9, 8, *BOX, seed=0))
    for kw in (dict(max_trials=0), dict(delta_min=0.0), dict(delta_min=1.0, delta_max=0.5)):
        with pytest.raises(SPError):
            P.newton_hookstep(u.clone(), max_newton=1, max_krylov=5, **kw)


@pytest.mark.parametrize("case", [((32, 33, 32), 400.0, 10.0), ((8, 97, 8), 1000.0, 100.0),
                                  ((8, 129, 8), 400.0, 1.0), ((12, 21, 24), 1000.0, 1.0)])
def test_device_build_equals_host_build(case):
    """The advected operators built on the device (one workgroup per mode,
    double-double refinement) against the host construction (long-double
    refinement): both are refined to about one rounding of the exact
    operator, so the steps and Jacobian actions they give agree to 1e-13.
    ny = 97 and 129 have more right-hand sides (3 (N - 1) = 285, 381) than
    the 256 threads of a workgroup."""
    import torch
    from paper_1804_05087_amd import Plan
    dims, re, dt = case
    say("advected device vs host build", dims, re, dt)
    u = to_dev(synth.perturbation_field(*dims, *BOX, seed=2, energy=0.05))
    du = to_dev(synth.random_admissible(*dims, *BOX, seed=3))
    out = {}
    for host in (False, True):
        P = Plan(*dims, *BOX, re, dt)
        P.set_advection(True, host_build=host)
        out[host] = (to_np(P.befe_step(u)), to_np(P.jvp(u, du, SP_OP_RESIDUAL)))
        torch.cuda.synchronize()
    e_phi = rel(out[False][0], out[True][0])
    e_jvp = rel(out[False][1], out[True][1])
    say("phi", e_phi, "jvp", e_jvp)
    assert e_phi < 1e-13 and e_jvp < 1e-13


def test_advection_mode_value_rejected():
    from paper_1804_05087_amd import Plan
    dims = (8, 9, 8)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    assert P.lib.sp_plan_set_advection(P.h, 3) != 0
    assert P.lib.sp_plan_set_advection(P.h, -1) != 0
