"""Batched evaluations (sp_befe_step_batch, sp_jvp_lin_batch): members run the
unchanged pipeline on their own intermediates and streams, so every result
equals the single call's bit for bit, and the argument contract holds."""
import numpy as np
import pytest

from gpu_util import BOX, say, to_dev
from paper_1804_05087_amd import SP_MIXED, SP_OP_PHI, SP_OP_RESIDUAL, SPError, synth

pytestmark = pytest.mark.gpu


def _fields(dims, count, seed0):
    import torch
    return torch.stack([to_dev(synth.perturbation_field(*dims, *BOX, seed=seed0 + i, energy=0.02))
                        for i in range(count)]).contiguous()


@pytest.mark.parametrize("dims,streams,precision,count", [
    ((16, 17, 16), 3, 0, 7), ((12, 21, 24), 8, 0, 7), ((16, 17, 16), 4, SP_MIXED, 7),
    ((16, 17, 16), 3, 0, 37),        # more members than streams, several rounds
    ((48, 65, 48), 2, 0, 18),        # the full grid
    ((48, 65, 48), 3, SP_MIXED, 17),
    ((18, 17, 16), 3, 0, 7)])        # x length 27: the LDS transform path
def test_batch_equals_single_calls(dims, streams, precision, count):
    import torch
    from paper_1804_05087_amd import Plan
    say("batch", dims, streams, precision, count)
    P = Plan(*dims, *BOX, 400.0, 10.0, precision=precision)
    u = _fields(dims, count, 10)
    out = P.befe_step_batch(u, streams=streams)
    for i in range(u.shape[0]):
        assert torch.equal(out[i], P.befe_step(u[i].contiguous())), i
    P.linearize(u[0].contiguous())
    du = _fields(dims, min(count, 19), 30)
    for op in (SP_OP_PHI, SP_OP_RESIDUAL):
        jb = P.jvp_lin_batch(du, op, streams=streams)
        for i in range(du.shape[0]):
            assert torch.equal(jb[i], P.jvp_lin(du[i].contiguous(), op)), (op, i)
    # an empty batch does nothing
    empty = torch.empty((0,) + P.shape, dtype=torch.complex128, device=P.device)
    assert P.befe_step_batch(empty).shape[0] == 0


def test_batch_rejects_bad_arguments():
    import torch
    from paper_1804_05087_amd import Plan
    dims = (8, 9, 8)
    P = Plan(*dims, *BOX, 400.0, 1.0)
    u = _fields(dims, 3, 0)
    for streams in (0, 9):
        with pytest.raises(SPError):
            P.befe_step_batch(u, streams=streams)
    with pytest.raises(SPError):
        P.befe_step_batch(u, out=u)  # in place is not allowed
    with pytest.raises(SPError):
        P.jvp_lin_batch(u)  # no base state
    P.linearize(u[0].contiguous())
    P.set_steps(3)
    P.linearize(u[0].contiguous())
    with pytest.raises(SPError):
        P.jvp_lin_batch(u, SP_OP_RESIDUAL)
    P.jvp_lin_batch(u, SP_OP_PHI)  # the one-step action is still allowed
    P.set_steps(1)
    P.set_advection(True)
    with pytest.raises(SPError):
        P.befe_step_batch(u)
    torch.cuda.synchronize()
