"""GPU adjoint: the VJP of Phi_dt against the oracle, dot-product identities,
the dense Jacobian transpose, and autograd gradients against central finite
differences (the adjoint workload: 32x33x32, Re = 400, dt = 100; dense
Jacobian on 8x9x8)."""
import numpy as np
import pytest

from gpu_util import BOX, rel, say, to_dev, to_np
from oracle.befe import Befe
from oracle.grid import Grid
from paper_1804_05087_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12
# 16x17x16, 32x33x32, 16x17x32 and 32x25x16 (nx a multiple of 16) take the
# adjoint z-line kernel that forms the inverse x transforms of its three
# fields itself; the others run the separate inverse x kernel
GRIDS = [(8, 9, 8, 400.0, 100.0), (16, 17, 16, 400.0, 100.0), (12, 21, 24, 1000.0, 1.0),
         (32, 33, 32, 400.0, 100.0), (16, 17, 32, 400.0, 100.0), (32, 25, 16, 1000.0, 10.0),
         (8, 97, 8, 400.0, 100.0), (8, 129, 8, 1000.0, 10.0), (8, 64, 8, 1000.0, 10.0)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


_cache = {}


def _setup(dims, re, dt):
    from paper_1804_05087_amd import Plan
    key = (dims, re, dt)
    if key not in _cache:
        g = Grid(*dims, *BOX)
        _cache[key] = (g, Befe(g, re, dt), Plan(*dims, *BOX, re, dt))
    return _cache[key]


def _tol(case):
    """1e-12, or machine epsilon times the largest condition number of the
    per-mode tau systems where that is larger (tall grids): the oracle's refined
    solve is accurate to ~1e-15, while a direct FP64 solve of the same system is
    only backward stable, so adjoint directions that probe the ill-conditioned
    high Chebyshev coefficients may differ by up to eps * cond."""
    import math
    from oracle.stokes import mode_matrix
    nx, ny, nz, re, dt = case
    kx, kz = 2 * math.pi / BOX[0], 2 * math.pi / BOX[1]
    cond = max(np.linalg.cond(mode_matrix(ny - 1, a, b, re, 1.0 / dt))
               for a, b in ((kx, 0.0), (0.0, kz)))
    return max(TOL, np.finfo(float).eps * cond)


@pytest.mark.parametrize("case", GRIDS)
def test_vjp_parity(torch_mod, case):
    from paper_1804_05087_amd import SP_OP_PHI, SP_OP_RESIDUAL
    nx, ny, nz, re, dt = case
    say("vjp parity", case)
    g, B, P = _setup((nx, ny, nz), re, dt)
    u = synth.perturbation_field(nx, ny, nz, *BOX, seed=1)
    w = synth.random_spectral(nx, ny, nz, seed=3)
    P.linearize(to_dev(u))
    tol = _tol(case)
    for op, name in ((SP_OP_PHI, "phi"), (SP_OP_RESIDUAL, "residual")):
        ref = B.vjp(u, w, name)
        got = to_np(P.vjp_lin(to_dev(w), op))
        assert rel(got, ref) < tol, (name, rel(got, ref), tol)


@pytest.mark.parametrize("case", GRIDS)
def test_vjp_dot_product(torch_mod, case):
    from paper_1804_05087_amd import SP_OP_RESIDUAL
    torch = torch_mod
    nx, ny, nz, re, dt = case
    say("dot test", case)
    g, B, P = _setup((nx, ny, nz), re, dt)
    u = to_dev(synth.perturbation_field(nx, ny, nz, *BOX, seed=2))
    v = to_dev(synth.random_spectral(nx, ny, nz, seed=5))
    w = to_dev(synth.random_spectral(nx, ny, nz, seed=6))
    P.linearize(u)
    pw, pv = P.pack(w), P.pack(v)
    pjv, pjtw = P.pack(P.jvp_lin(v, SP_OP_RESIDUAL)), P.pack(P.vjp_lin(w, SP_OP_RESIDUAL))
    lhs = torch.dot(pw, pjv).item()
    rhs = torch.dot(pjtw, pv).item()
    # rounding errors of the two products scale with the vectors' norms (the
    # Cauchy-Schwarz bound of each inner product), not with the inner product,
    # which may cancel far below it for white-noise vectors
    scale = (torch.linalg.norm(pw) * torch.linalg.norm(pjv) +
             torch.linalg.norm(pjtw) * torch.linalg.norm(pv)).item()
    tol = _tol(case)
    say("dot test", case, "difference / scale", abs(lhs - rhs) / scale, "tol", tol)
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs, scale, tol)


def test_dense_jacobian_transpose_8x9x8(torch_mod):
    torch = torch_mod
    from paper_1804_05087_amd import SP_OP_PHI
    dims = (8, 9, 8)
    say("dense J 8x9x8")
    g, B, P = _setup(dims, 400.0, 100.0)
    u_np = synth.perturbation_field(*dims, *BOX, seed=0)
    P.linearize(to_dev(u_np))
    n = P.packed_n
    assert n == 1323
    J = torch.empty((n, n), dtype=torch.float64, device=P.device)
    JT = torch.empty((n, n), dtype=torch.float64, device=P.device)
    e = torch.zeros(n, dtype=torch.float64, device=P.device)
    for k in range(n):
        e.zero_()
        e[k] = 1.0
        ek = P.unpack(e)
        J[:, k] = P.pack(P.jvp_lin(ek, SP_OP_PHI))
        JT[:, k] = P.pack(P.vjp_lin(ek, SP_OP_PHI))
    J = J.cpu().numpy()
    JT = JT.cpu().numpy()
    scale = np.abs(J).max()
    assert np.abs(JT - J.T).max() < 1e-13 * scale
    # columns against the oracle's JVP
    from oracle import pack as opack
    rng = np.random.default_rng(0)
    for k in rng.choice(n, 10, replace=False):
        ek = np.zeros(n)
        ek[k] = 1.0
        col = opack.pack(B.jvp(u_np, opack.unpack(ek, g)), g)
        assert np.abs(col - J[:, k]).max() < 1e-13 * scale
    # J_Phi maps onto the admissible subspace (2N-4 per k != 0 mode, 2(N-1) for (0,0))
    N = g.N
    m = (2 * N - 4) * ((g.nx - 1) * (g.nz - 1) - 1) + 2 * (N - 1)
    s = np.linalg.svd(J, compute_uv=False)
    assert int(np.sum(s > 1e-10 * s[0])) == m


def test_autograd_gradient_vs_central_differences(torch_mod):
    """Gradient of L(x) = 1/2 ||Phi(x) - x||^2 (packed vectors) through
    PhiFunction against central differences, h = 1e-6, 20 seeded directions."""
    torch = torch_mod
    from paper_1804_05087_amd import PhiFunction
    dims = (32, 33, 32)
    say("autograd FD 32x33x32")
    g, B, P = _setup(dims, 400.0, 100.0)
    u = to_dev(synth.perturbation_field(*dims, *BOX, seed=0))
    x = P.pack(u).clone().requires_grad_(True)
    loss = 0.5 * torch.sum((PhiFunction.apply(x, P) - x) ** 2)
    loss.backward()
    grad = x.grad.detach()

    def L(xx):
        with torch.no_grad():
            return 0.5 * torch.sum((PhiFunction.apply(xx, P) - xx) ** 2).item()

    gen = torch.Generator(device="cpu").manual_seed(0)
    h = 1e-6
    worst = 0.0
    for _ in range(20):
        d = torch.randn(P.packed_n, generator=gen, dtype=torch.float64).to(P.device)
        d /= torch.linalg.norm(d)
        fd = (L(x.detach() + h * d) - L(x.detach() - h * d)) / (2 * h)
        an = torch.dot(grad, d).item()
        worst = max(worst, abs(fd - an) / (abs(an) + 1e-30))
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9 * loss.item(), (fd, an)
    say("autograd worst rel FD mismatch", worst)


def test_autograd_gradient_mixed_precision(torch_mod):
    """The FP32 variant of the adjoint workload: the gradient of
    L(x) = 1/2 ||Phi(x) - x||^2 through PhiFunction on a mixed-precision plan
    (FP32 transforms, products and y-contractions; FP64 solves) against the FP64
    plan's gradient and against central differences of the FP64 loss (h = 1e-6,
    20 seeded directions). FP32 rounding (unit 6e-8) amplified by the transform
    and solve chain bounds the gap at ~1e-6 of the gradient's norm."""
    torch = torch_mod
    from paper_1804_05087_amd import SP_MIXED, Plan, PhiFunction
    dims = (32, 33, 32)
    say("autograd mixed 32x33x32")
    g, B, P = _setup(dims, 400.0, 100.0)
    PM = Plan(*dims, *BOX, 400.0, 100.0, precision=SP_MIXED)
    u = to_dev(synth.perturbation_field(*dims, *BOX, seed=0))
    x0 = P.pack(u).clone()

    def grad_of(plan):
        x = x0.clone().requires_grad_(True)
        loss = 0.5 * torch.sum((PhiFunction.apply(x, plan) - x) ** 2)
        loss.backward()
        return x.grad.detach(), loss.item()

    g64, loss64 = grad_of(P)
    g32, loss32 = grad_of(PM)
    gn = torch.linalg.norm(g64).item()
    e_grad = torch.linalg.norm(g32 - g64).item() / gn
    say("mixed gradient: rel error vs FP64", e_grad, "loss rel diff", abs(loss32 - loss64) / loss64)
    assert e_grad < 2e-5
    assert abs(loss32 - loss64) <= 2e-5 * loss64

    def L(xx):
        with torch.no_grad():
            return 0.5 * torch.sum((PhiFunction.apply(xx, P) - xx) ** 2).item()

    gen = torch.Generator(device="cpu").manual_seed(1)
    h = 1e-6
    worst = 0.0
    for _ in range(20):
        d = torch.randn(P.packed_n, generator=gen, dtype=torch.float64).to(P.device)
        d /= torch.linalg.norm(d)
        fd = (L(x0 + h * d) - L(x0 - h * d)) / (2 * h)
        an = torch.dot(g32, d).item()
        worst = max(worst, abs(fd - an) / gn)
        assert abs(fd - an) <= 2e-5 * gn, (fd, an, gn)
    say("mixed gradient: worst FD mismatch / ||grad||", worst)
