"""The residual Jacobian action J_r du = (J_Phi du - du)/dt formed by the solve
kernel itself (Sec. 2, eq. Gstokes and after eq. factor2): it must equal the
Phi action combined on the host, within rounding, and be written in the exact
Hermitian form that the packed space assumes (the m_z = 0 plane at -m_x the
conjugate of +m_x, the (0,0) mode real, Nyquist entries zero)."""
import numpy as np
import pytest

from gpu_util import BOX, say, to_dev, to_np
from paper_1804_05087_amd import synth

pytestmark = pytest.mark.gpu

CASES = [(16, 17, 16, 400.0, 100.0), (12, 20, 16, 400.0, 10.0), (48, 65, 48, 1000.0, 100.0)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _check_hermitian_form(a, nx, nz):
    # a: [3][nx][nz/2+1][ny] complex
    nzh = nz // 2 + 1
    assert np.all(a[:, nx // 2, :, :] == 0) and np.all(a[:, :, nzh - 1, :] == 0)
    assert np.all(a[:, 0, 0, :].imag == 0)
    for i in range(1, nx // 2):
        assert np.array_equal(a[:, nx - i, 0, :], np.conj(a[:, i, 0, :])), i


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_residual_action_formed_in_the_solve(torch_mod, case, mixed):
    from paper_1804_05087_amd import SP_FP64, SP_MIXED, SP_OP_PHI, SP_OP_RESIDUAL, Plan
    nx, ny, nz, re, dt = case
    say("residual form", case, "mixed" if mixed else "fp64")
    P = Plan(nx, ny, nz, *BOX, re, dt, precision=SP_MIXED if mixed else SP_FP64)
    u = synth.perturbation_field(nx, ny, nz, *BOX, seed=3)
    P.linearize(to_dev(u))
    for du in (synth.random_admissible(nx, ny, nz, *BOX, seed=4),
               synth.random_spectral(nx, ny, nz, seed=5)):
        jr = to_np(P.jvp_lin(to_dev(du), SP_OP_RESIDUAL))
        jp = to_np(P.jvp_lin(to_dev(du), SP_OP_PHI))
        _check_hermitian_form(jr, nx, nz)
        want = (jp - du) / dt
        # compared where the Hermitian form keeps the values computed by the
        # mode itself: every mode except the m_z = 0 modes at negative m_x
        keep = np.ones((nx, nz // 2 + 1), bool)
        keep[nx // 2 + 1:, 0] = False
        keep[nx // 2, :] = False
        keep[:, nz // 2] = False
        want[:, 0, 0, :] = want[:, 0, 0, :].real
        scale = (np.linalg.norm(jp) + np.linalg.norm(du)) / dt
        err = np.linalg.norm((jr - want)[:, keep, :])
        assert err < 1e-14 * scale, err / scale
