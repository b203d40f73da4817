"""GPU projection onto the shift-reflect invariant subspace (EQ1's symmetry
group, Sec. 3.3) against the oracle's composition of the elementary
symmetries, and a Newton solve confined to the subspace."""
import math

import numpy as np
import pytest

from gpu_util import BOX, rel, say, to_dev, to_np
from oracle import krylov
from oracle import symmetry as sym
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims", [(8, 9, 8), (12, 21, 24), (16, 17, 16)])
def test_projection_matches_oracle(dims):
    from paper_1804_05087_amd import Plan
    g = Grid(*dims, *BOX)
    P = Plan(*dims, *BOX, 400.0, 1.0)
    a = synth.random_spectral(*dims, seed=4)
    got = to_np(P.symmetrize(to_dev(a)))
    ref = sym.project(g, a)
    say("symmetrize", dims, rel(got, ref))
    assert rel(got, ref) < 1e-13
    twice = to_np(P.symmetrize(to_dev(got)))
    assert rel(twice, got) < 1e-15


def test_newton_in_the_subspace():
    from paper_1804_05087_amd import Plan
    dims = (8, 9, 8)
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, 100.0)
    P = Plan(*dims, *BOX, 400.0, 100.0)
    P.set_symmetry(True)
    u0 = sym.project(g, synth.perturbation_field(*dims, *BOX, seed=0, energy=1e-2))
    _, ref = krylov.newton_hook_befe(B, u0, 1e-10, 3, 15, 1e-6)
    u = to_dev(u0)
    rep = P.newton_hookstep(u, max_newton=3, max_krylov=15, gmres_rtol=1e-6, newton_tol=1e-10)
    say("gpu", rep["res_norm"], rep["krylov"], "ref", ref["res_norm"], ref["krylov"])
    assert rep["krylov"] == ref["krylov"]
    for x, y in zip(rep["res_norm"], ref["res_norm"]):
        assert abs(x - y) <= 1e-8 * y
    out = to_np(u)
    assert rel(sym.project(g, out), out) < 1e-13
