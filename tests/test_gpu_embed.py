"""Periodic embedding commutes with Phi on the GPU: for a field a of an
Lx x Lz box, Phi of the 2Lx x 2Lz box applied to synth.embed_periodic(a) is
the embedding of Phi(a) (the product of fields with even modes only has even
modes only, and the 3/2 padding keeps the same modes), so a root of the small
box is a root of the large one. This is what the large-grid Newton solve at
96x97x96 relies on (the 2pi x pi box's root checked on the 4pi x 2pi grid).
Checked in FP64 and in the mixed path, on two grid pairs."""
import math

import numpy as np
import pytest

from gpu_util import rel, say, to_dev, to_np
from paper_1804_05087_amd import SP_FP64, SP_MIXED, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [(SP_FP64, 1e-13), (SP_MIXED, 1e-5)])
@pytest.mark.parametrize("small", [(8, 17, 8), (16, 33, 16)])
def test_embedding_commutes_with_phi(small, prec, tol):
    from paper_1804_05087_amd import Plan
    nx, ny, nz = small
    lx, lz = 2 * math.pi, math.pi
    say("embed", small, prec)
    Ps = Plan(nx, ny, nz, lx, lz, 800.0, 100.0)
    Pb = Plan(2 * nx, ny, 2 * nz, 2 * lx, 2 * lz, 800.0, 100.0)
    Ps.set_precision(prec)
    Pb.set_precision(prec)
    a = synth.perturbation_field(nx, ny, nz, lx, lz, seed=4, energy=5e-2)
    phi_s = to_np(Ps.befe_step(to_dev(a)))
    phi_b = to_np(Pb.befe_step(to_dev(synth.embed_periodic(a, 2, 2))))
    want = synth.embed_periodic(phi_s, 2, 2)
    assert rel(phi_b, want) < tol, rel(phi_b, want)
    # and the residual norms agree (the volume-normalised norm of a periodic extension)
    _, rs = Ps.residual(to_dev(a), norm=True)
    _, rb = Pb.residual(to_dev(synth.embed_periodic(a, 2, 2)), norm=True)
    assert abs(rs - rb) <= tol * rs, (rs, rb)
