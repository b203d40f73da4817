"""Error paths on the device, through the C ABI: a state holding NaN or Inf
makes the residual norm non-finite, and sp_residual (with a host norm) and
both Newton drivers return SP_ERR_NONFINITE instead of iterating on it. The
kernels have no data-dependent loops, so non-finite values only propagate."""
import math

import numpy as np
import pytest

from gpu_util import BOX, say, to_dev
from paper_1804_05087_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("bad", [math.nan, math.inf])
def test_nonfinite_state_reports_nonfinite(torch_mod, bad):
    from paper_1804_05087_amd import Plan
    from paper_1804_05087_amd._lib import SP_ERR_NONFINITE, SPError
    dims = (16, 17, 16)
    say("non-finite state", bad)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    u = synth.perturbation_field(*dims, *BOX, seed=0)
    u[1, 3, 2, 4] = complex(bad, 0.0)
    with pytest.raises(SPError) as e:
        P.residual(to_dev(u), norm=True)
    assert e.value.status == SP_ERR_NONFINITE
    with pytest.raises(SPError) as e:
        P.norm(to_dev(u))
    assert e.value.status == SP_ERR_NONFINITE
    for drive in (P.newton_gmres, P.newton_hookstep):
        x = to_dev(u)
        with pytest.raises(SPError) as e:
            drive(x, max_newton=3, max_krylov=10)
        assert e.value.status == SP_ERR_NONFINITE, drive.__name__
    # the plan stays usable after the error
    good = synth.perturbation_field(*dims, *BOX, seed=0)
    _, nrm = P.residual(to_dev(good), norm=True)
    assert np.isfinite(nrm) and nrm > 0
