"""Mixed precision: FP32 transforms/products/y-contractions with the FP64
implicit solve. The error of each result against the FP64 oracle is stated
(printed) and bounded; FP32 rounding (unit 6e-8) amplified by the transform
and solve chain is expected around 1e-7..1e-6 relative."""
import pytest

from gpu_util import BOX, rel, say, to_dev, to_np
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

pytestmark = pytest.mark.gpu
BOUND = 2e-5


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("case", [(16, 17, 16, 400.0, 100.0), (32, 33, 32, 400.0, 100.0),
                                  (48, 65, 48, 1000.0, 100.0)])
def test_mixed_errors_against_fp64_oracle(torch_mod, case):
    from paper_1804_05087_amd import SP_MIXED, SP_OP_PHI, Plan
    nx, ny, nz, re, dt = case
    dims = (nx, ny, nz)
    g = Grid(*dims, *BOX)
    small = nx <= 32
    B = Befe(g, re, dt) if small else Befe(g, re, dt, modes=[(0, 0), (1, 0), (0, 1), (3, 2)])
    P = Plan(*dims, *BOX, re, dt, precision=SP_MIXED)
    u = synth.perturbation_field(*dims, *BOX, seed=0)
    du = synth.random_admissible(*dims, *BOX, seed=1)
    w = synth.random_spectral(*dims, seed=2)
    n_ref = B.nonlinear(u)
    phi = to_np(P.befe_step(to_dev(u)))
    if small:
        e_phi = rel(phi, B.phi(u))
        P.linearize(to_dev(u))
        e_jvp = rel(to_np(P.jvp_lin(to_dev(du), SP_OP_PHI)), B.jvp(u, du))
        e_vjp = rel(to_np(P.vjp_lin(to_dev(w), SP_OP_PHI)), B.vjp(u, w))
        say("mixed errors", case, "phi", e_phi, "jvp", e_jvp, "vjp", e_vjp)
        assert e_phi < BOUND and e_jvp < BOUND and e_vjp < BOUND
    else:
        ref = B.phi(u)
        modes = [(0, 0), (1, 0), (0, 1), (3, 2)]
        import numpy as np
        idx = tuple(np.array(modes).T)
        e_phi = rel(phi[:, idx[0], idx[1]], ref[:, idx[0], idx[1]])
        say("mixed errors", case, "phi (sampled modes)", e_phi)
        assert e_phi < BOUND
