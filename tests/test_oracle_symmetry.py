"""Pins of the shift-reflect symmetry subspace (EQ1's group, Sec. 3.3)."""
import math

import numpy as np

from oracle import symmetry as sym
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)


def test_projector_and_group():
    dims = (8, 13, 8)
    g = Grid(*dims, *BOX)
    a = synth.random_spectral(*dims, seed=1)
    for s in (sym.s1, sym.s2):
        assert np.abs(s(g, s(g, a)) - a).max() < 1e-13          # involutions (phases exp(i pi m) round)
    p = sym.project(g, a)
    assert np.abs(sym.project(g, p) - p).max() < 1e-13           # idempotent
    assert np.abs(sym.s1(g, p) - p).max() < 1e-13                # invariant under s1
    assert np.abs(sym.s2(g, p) - p).max() < 1e-13                # and s2
    # s1 s2 = s2 s1 (the group is abelian)
    assert np.abs(sym.s1(g, sym.s2(g, a)) - sym.s2(g, sym.s1(g, a))).max() < 1e-13
    # the projection removes the translation directions of an invariant field
    u = sym.project(g, synth.perturbation_field(*dims, *BOX, seed=2))
    du_dx = u * (1j * g.kx())[None, :, None, None]
    assert np.abs(sym.project(g, du_dx)).max() < 1e-13 * np.abs(du_dx).max()


def test_phi_preserves_the_subspace():
    dims = (8, 13, 8)
    g = Grid(*dims, *BOX)
    B = Befe(g, 400.0, 10.0)
    u = sym.project(g, synth.perturbation_field(*dims, *BOX, seed=3, energy=0.05))
    phi = B.phi(u)
    assert np.abs(sym.project(g, phi) - phi).max() < 1e-14 * np.abs(phi).max()
    lam = synth.laminar_field(*dims)
    assert np.abs(sym.project(g, lam) - lam).max() < 1e-15      # laminar flow is invariant
