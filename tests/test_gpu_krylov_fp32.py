"""Newton-GMRES with the Krylov basis stored in FP32 (krylov_fp32 = 1): the
orthogonalisation reads and writes half the bytes, while the dot products,
the GMRES scalars, the residual and the Newton update stay FP64.

Bar, from the arithmetic. Each stored basis entry carries a relative rounding
error of at most 2^-24 = 6e-8, and the delayed CGS2 pass re-orthogonalises
every candidate against the stored vectors, so the basis stays orthonormal to
a few times 1e-7 and the step du = Q y is accurate to about 1e-6 relative. At
gmres_rtol = 1e-3 the residual after a step is about 1e-3 ||r||, so its
relative difference from the FP64 path is at most about 1e-6 / 1e-3 = 1e-3:
the residual histories are compared at 1e-2, the Krylov counts exactly (a
count changes only if the GMRES estimate lands within 1e-6 of the threshold).
Converged roots are compared at 1e-8 relative (both residuals < 1e-10).
"""
import numpy as np
import pytest

from gpu_util import BOX, say, to_dev
from oracle import krylov
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

pytestmark = pytest.mark.gpu


def test_short_newton_matches_oracle():
    from paper_1804_05087_amd import Plan
    dims = (8, 9, 8)
    say("krylov fp32 against the oracle, 8x9x8")
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, 100.0)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    u0 = synth.perturbation_field(*dims, *BOX, seed=0)
    _, ref = krylov.newton_befe(B, u0, 1e-10, 3, 15, 1e-3)
    u = to_dev(u0)
    rep = P.newton_gmres(u, max_newton=3, max_krylov=15, gmres_rtol=1e-3, newton_tol=1e-10,
                         krylov_fp32=True)
    say("gpu", rep["res_norm"], rep["krylov"], "oracle", ref["res_norm"], ref["krylov"])
    assert rep["krylov"] == ref["krylov"]
    assert len(rep["res_norm"]) == len(ref["res_norm"])
    assert abs(rep["res_norm"][0] - ref["res_norm"][0]) <= 1e-12 * ref["res_norm"][0]
    for a, b in zip(rep["res_norm"][1:], ref["res_norm"][1:]):
        assert abs(a - b) <= 1e-2 * b


@pytest.mark.parametrize("hook", [False, True])
def test_root_matches_fp64_basis(hook):
    import torch
    from paper_1804_05087_amd import Plan
    dims = (32, 33, 32)
    say("krylov fp32 against the fp64 basis, 32x33x32, hookstep", hook)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    u0 = to_dev(synth.perturbation_field(*dims, *BOX, seed=0, energy=1e-6))
    out = {}
    for f32 in (False, True):
        u = u0.clone()
        kw = dict(max_newton=16, max_krylov=200, gmres_rtol=1e-3, newton_tol=1e-10,
                  krylov_fp32=f32)
        rep = P.newton_hookstep(u, **kw) if hook else P.newton_gmres(u, **kw)
        say("fp32" if f32 else "fp64", rep["converged"], rep["krylov"], rep["res_norm"][-1])
        assert rep["converged"]
        assert rep["res_norm"][-1] < 1e-10
        out[f32] = (u, rep)
    (ua, ra), (ub, rb) = out[False], out[True]
    d = P.norm((ub - ua).contiguous()) / P.norm(ua)
    say("root distance", d)
    assert d < 1e-8
    assert abs(rb["total_krylov"] - ra["total_krylov"]) <= 0.1 * ra["total_krylov"]
    torch.cuda.synchronize()


def test_invalid_flag_rejected():
    from paper_1804_05087_amd import Plan, SPError
    dims = (8, 9, 8)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    u = to_dev(synth.perturbation_field(*dims, *BOX, seed=0))
    u_before = u.clone()
    with pytest.raises(SPError):
        P.newton_gmres(u, max_newton=1, max_krylov=5, krylov_fp32=2)
    assert np.array_equal(u.cpu().numpy(), u_before.cpu().numpy())
