"""GPU parity of the differentiation path: the adjoint solve, the link-gradient
kernels against the oracle's chain rule, and the autograd Function against
FP64 central finite differences on the 16^3 x 32 lattice (kappa 0.13, c_SW 1.0,
loss L = Re<eta, D^-1 b>).

Tolerances: the gradient kernels are FP64 and agree with the oracle to
1e-12 relative; directional derivatives agree with central differences of
step 1e-6 (FP64 solves to 1e-13) to 1e-5 relative (the finite-difference
budget: truncation ~h^2, solve noise ~1e-13 / h).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (2, 2, 2, 2), (4, 2, 6, 4)])
def test_link_grad_kernel_matches_oracle(dims, csw):
    say("link_grad", dims, csw)
    kappa = 0.13
    U = synth.random_links(dims, 0.3, 401)
    lam = synth.gaussian_source(dims, 402)
    x = synth.gaussian_source(dims, 403)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    G = host(lat.link_grad(dev(lam), dev(x), kappa, csw))
    ref = oracle.link_grad(U, lam, x, kappa, csw)
    assert rel(G, ref) < 1e-12
    Gh = host(lat.link_grad(dev(lam), dev(x), kappa, csw, include_clover=False))
    assert rel(Gh, oracle.link_grad(U, lam, x, kappa, csw, include_clover=False)) < 1e-12


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP64])
def test_adjoint_solve_matches_oracle(inner):
    dims = (8, 8, 8, 8)
    kappa, csw = 0.13, 1.0
    say("adjoint", inner)
    U = synth.random_links(dims, 0.3, 411)
    eta = synth.gaussian_source(dims, 412)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    lam, info = lat.solve(dev(eta), kappa, csw, 1e-12, inner_prec=inner, adjoint=1)
    F = oracle.clover_field(U, dims, kappa, csw)
    ref = oracle.adjoint_solve(U, F, kappa, eta, tol=1e-13)
    assert rel(host(lam), ref) < 1e-10


DIMS5 = (16, 16, 16, 32)
KAPPA5, CSW5 = 0.13, 1.0


@pytest.fixture(scope="module")
def case5():
    U = synth.random_links(DIMS5, 0.3, 1005)
    eta = synth.gaussian_source(DIMS5, 2005)
    b = synth.gaussian_source(DIMS5, 3005)
    lat = wc.Lattice(DIMS5)
    return lat, U, eta, b


def test_autograd_matches_oracle_gradient(case5):
    lat, U, eta, b = case5
    say("autograd vs oracle", DIMS5)
    Ud = dev(U).requires_grad_(True)
    bd = dev(b).requires_grad_(True)
    etad = dev(eta)
    x = wc.solve(lat, bd, Ud, KAPPA5, CSW5, tol=1e-12)
    L = torch.real(torch.vdot(etad.reshape(-1), x.reshape(-1)))
    L.backward()
    # oracle: lam and x from its own solves, gradient by its own chain rule
    F = oracle.clover_field(U, DIMS5, KAPPA5, CSW5)
    x_ref, _, _ = oracle.solve(U, F, KAPPA5, b, tol=1e-13)
    lam_ref = oracle.adjoint_solve(U, F, KAPPA5, eta, tol=1e-13)
    assert rel(host(x), x_ref) < 1e-10
    assert rel(host(bd.grad), lam_ref) < 1e-10
    G_ref = oracle.link_grad(U, lam_ref, x_ref, KAPPA5, CSW5)
    assert rel(host(Ud.grad), G_ref) < 1e-9


def _moved(U, X, h):
    # exp(i h X) U to fourth order in h; the remainder (h |X|)^5 / 120 is far below FP64 rounding
    A = 1j * h * X
    A2 = A @ A
    E = torch.eye(3, dtype=U.dtype, device=U.device) + A + A2 / 2 + A2 @ A / 6 + A2 @ A2 / 24
    return (E @ U).contiguous()


def test_fd_64_directions(case5):
    lat, U, eta, b = case5
    say("fd 64 directions", DIMS5)
    Ud = dev(U).requires_grad_(True)
    bd = dev(b)
    etad = dev(eta)
    x = wc.solve(lat, bd, Ud, KAPPA5, CSW5, tol=1e-13, inner_prec=wc.FP64)
    L = torch.real(torch.vdot(etad.reshape(-1), x.reshape(-1)))
    L.backward()
    G = Ud.grad.detach()
    Ub = Ud.detach()
    h = 1e-6
    worst = 0.0
    for k in range(64):
        X = dev(synth.random_hermitian_traceless(U.shape[:-2], synth.rng(5000 + k)))
        vals = []
        for s in (+1, -1):
            Uh = _moved(Ub, X, s * h)
            lat.load_links(Uh)
            xh, info = lat.solve(bd, KAPPA5, CSW5, 1e-13, inner_prec=wc.FP64)
            vals.append(float(torch.real(torch.vdot(etad.reshape(-1), xh.reshape(-1)))))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(torch.real(torch.vdot(G.reshape(-1), (1j * X @ Ub).reshape(-1))))
        err = abs(fd - an) / max(abs(an), 1e-30)
        worst = max(worst, err)
        if k < 4 or err > 1e-5:
            say("dir", k, "fd", fd, "grad", an, "rel", err)
        assert err < 1e-5, (k, fd, an)
    say("worst relative error over 64 directions", worst)
