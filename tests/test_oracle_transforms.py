"""Pins for the oracle's transforms, packing and dealiased product (CPU)."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C
from numpy.polynomial import legendre as Leg

from oracle import cheb, fourier, pack
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_synthesis_matches_chebval(N):
    rng = np.random.default_rng(N)
    a = rng.standard_normal(N + 1)
    y = cheb.points(N)
    assert np.allclose(cheb.synthesis(N) @ a, C.chebval(y, a), atol=1e-13)


@pytest.mark.parametrize("N", [4, 16, 64, 96])
def test_analysis_inverts_synthesis(N):
    I = cheb.analysis(N) @ cheb.synthesis(N)
    assert np.abs(I - np.eye(N + 1)).max() < 1e-13


@pytest.mark.parametrize("N", [4, 9, 16, 33])
def test_derivative_matches_chebder(N):
    rng = np.random.default_rng(N)
    a = rng.standard_normal(N + 1)
    ref = np.zeros(N + 1)
    d = C.chebder(a)
    ref[: len(d)] = d
    assert np.allclose(cheb.derivative(N) @ a, ref, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("N", [4, 12, 20])
def test_gram_matches_quadrature(N):
    x, w = Leg.leggauss(2 * N + 4)
    V = np.stack([C.chebval(x, np.eye(N + 1)[n]) for n in range(N + 1)])
    ref = (V * w) @ V.T
    assert np.abs(cheb.gram(N) - ref).max() < 1e-13


def test_fft_roundtrip_and_single_mode():
    g = Grid(8, 5, 12, *BOX)
    a = synth.random_spectral(8, 5, 12, seed=3)
    p = fourier.to_physical(a, g)
    assert p.dtype == np.float64
    back = fourier.to_spectral(p, g)
    assert np.abs(back - a).max() < 1e-14
    # single mode closed form: a_(mx=2, mz=1) = c -> 2 Re(c e^{i(2 alpha x + gamma z)})
    b = g.zeros()[0]
    c = 0.3 - 0.7j
    b[2, 1, :] = c
    x, z = fourier.physical_grid(g)
    ref = 2 * np.real(c * np.exp(1j * (2 * g.alpha * x[:, None] + g.gamma * z[None, :])))
    got = fourier.to_physical(b, g)[:, :, 0]
    assert np.abs(got - ref).max() < 1e-14
    # negative m_x in the m_z = 0 plane
    b = g.zeros()[0]
    b[g.nx - 3, 0, :] = c
    b[3, 0, :] = np.conj(c)
    ref = 2 * np.real(c * np.exp(-1j * 3 * g.alpha * x[:, None])) + 0 * z[None, :]
    got = fourier.to_physical(b, g)[:, :, 0]
    assert np.abs(got - ref).max() < 1e-14


def test_pack_roundtrip_and_inner_product():
    g = Grid(8, 5, 6, *BOX)
    a = synth.random_spectral(8, 5, 6, seed=1)
    b = synth.random_spectral(8, 5, 6, seed=2)
    x = pack.pack(a, g)
    assert x.shape == (pack.packed_length(g),) == (3 * 5 * 7 * 5,)
    assert np.array_equal(pack.unpack(x, g), a)
    assert abs(pack.packed_dot(a, b, g) - np.dot(pack.pack(a, g), pack.pack(b, g))) < 1e-12


def _brute_product(u, g, T):
    """Exact Fourier convolution of u x curl(u) in x,z and collocation in y,
    truncated to the kept modes. O(modes^2) loops; tiny grids only."""
    B = Befe(g, 1.0, 1.0)
    w = B.curl(u)
    uv = cheb.apply_y(T, u)
    wv = cheb.apply_y(T, w)
    mx = g.mx()
    # expand to the full set of (m_x, m_z) with negative m_z by symmetry
    full_u, full_w = {}, {}
    valid = g.valid()
    for i in range(g.nx):
        for j in range(g.nzh):
            if not valid[i, j]:
                continue
            full_u[(mx[i], j)] = uv[:, i, j, :]
            full_w[(mx[i], j)] = wv[:, i, j, :]
            if j > 0:
                full_u[(-mx[i], -j)] = np.conj(uv[:, i, j, :])
                full_w[(-mx[i], -j)] = np.conj(wv[:, i, j, :])
    out = np.zeros((3, g.nx, g.nzh, g.ny), dtype=complex)
    for i in range(g.nx):
        for j in range(g.nzh):
            if not valid[i, j]:
                continue
            target = (mx[i], j)
            acc = np.zeros((3, g.ny), dtype=complex)
            for (p, q), a in full_u.items():
                key = (target[0] - p, target[1] - q)
                if key in full_w:
                    acc += np.cross(a, full_w[key], axis=0)
            out[:, i, j, :] = acc
    return out


@pytest.mark.parametrize("dims", [(4, 5, 4), (8, 9, 8), (6, 7, 8)])
def test_dealiased_product_equals_brute_force(dims):
    nx, ny, nz = dims
    g = Grid(nx, ny, nz, *BOX)
    u = synth.random_spectral(nx, ny, nz, seed=7)
    B = Befe(g, 1.0, 1.0)
    n_fast = B.nonlinear(u)
    T = cheb.synthesis(g.N)
    n_brute = cheb.apply_y(cheb.analysis(g.N), _brute_product(u, g, T))
    assert np.abs(n_fast - n_brute).max() < 1e-13 * max(1.0, np.abs(n_brute).max())
