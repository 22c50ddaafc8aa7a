"""Pins of the oracle's link gradient and adjoint solve.

The gradient code (chain rule through eq. 4 and the clover leaves) is checked
against central finite differences of quantities the other pins already fix:
the operator itself (g(U) = -Re<lam, D[U] x>, no solve involved) and the full
loss L = Re<eta, D^-1 b> with FP64 solves to 1e-14 (BiCGStab, pinned against dense
LU elsewhere).  Directions keep the links in
SU(3): U(h) = exp(i h X) U with X Gaussian traceless Hermitian on every link.
"""
import numpy as np
import pytest

import oracle
import synth


def tangent(U, seed):
    X = synth.random_hermitian_traceless(U.shape[:-2], synth.rng(seed))
    return X


def moved(U, X, h):
    return synth.expi_hermitian(h * X) @ U


def directional(G, X, U):
    # d/dh at h = 0 of a function of U(h) = exp(i h X) U is Re sum conj(G) (i X U)
    delta = 1j * X @ U
    return float(np.real(np.vdot(G.reshape(-1), delta.reshape(-1))))


def fd_richardson(f, U, X, h):
    """Central difference at h and h/2 combined to cancel the h^2 term."""
    d1 = (f(moved(U, X, h)) - f(moved(U, X, -h))) / (2 * h)
    d2 = (f(moved(U, X, h / 2)) - f(moved(U, X, -h / 2))) / h
    return (4 * d2 - d1) / 3


def g_of(U, dims, kappa, csw, lam, x):
    F = oracle.clover_field(U, dims, kappa, csw)
    return -float(np.real(np.vdot(lam.reshape(-1), oracle.apply_D(U, F, kappa, x).reshape(-1))))


@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 2, 4)])
def test_link_grad_matches_fd_of_operator(dims, csw):
    kappa = 0.13
    U = synth.random_links(dims, 0.3, 301)
    lam = synth.gaussian_source(dims, 302)
    x = synth.gaussian_source(dims, 303)
    G = oracle.link_grad(U, lam, x, kappa, csw, include_clover=True)
    for k in range(4):
        X = tangent(U, 310 + k)
        fd = fd_richardson(lambda Uh: g_of(Uh, dims, kappa, csw, lam, x), U, X, 1e-3)
        an = directional(G, X, U)
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (k, fd, an)


def test_clover_part_is_the_difference():
    # include_clover=False must equal the c_SW = 0 gradient, and the clover part alone
    # must match the FD of g with the hopping term removed (kappa c_SW varied via c_SW)
    dims = (4, 4, 4, 4)
    kappa = 0.13
    U = synth.random_links(dims, 0.3, 321)
    lam = synth.gaussian_source(dims, 322)
    x = synth.gaussian_source(dims, 323)
    G0 = oracle.link_grad(U, lam, x, kappa, 0.0, include_clover=True)
    Gh = oracle.link_grad(U, lam, x, kappa, 1.0, include_clover=False)
    assert np.abs(G0 - Gh).max() == 0.0
    G1 = oracle.link_grad(U, lam, x, kappa, 1.0, include_clover=True)
    Gc = G1 - Gh
    # g_clover(U) = -Re<lam, (F[U] - 1) x>
    def gc(Uh):
        F = oracle.clover_field(Uh, dims, kappa, 1.0)
        return -float(np.real(np.vdot(lam.reshape(-1), (oracle.site_apply(F, x) - x).reshape(-1))))
    X = tangent(U, 330)
    fd = fd_richardson(gc, U, X, 1e-3)
    an = directional(Gc, X, U)
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_adjoint_solve_is_dagger_solve():
    dims = (2, 2, 2, 2)
    kappa = 0.13
    U = synth.random_links(dims, 0.3, 341)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    eta = synth.gaussian_source(dims, 342)
    M = oracle.dense_matrix(U, F, kappa, dims)
    lam_dense = np.linalg.solve(M.conj().T, eta.reshape(-1)).reshape(eta.shape)
    lam = oracle.adjoint_solve(U, F, kappa, eta, tol=1e-14)
    assert np.linalg.norm(lam - lam_dense) / np.linalg.norm(lam_dense) < 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_full_loss_gradient_fd(dims):
    # L(U) = Re<eta, D[U]^-1 b>; gradient at lam = D^-dag eta, x = D^-1 b
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 351)
    eta = synth.gaussian_source(dims, 352)
    b = synth.gaussian_source(dims, 353)
    F = oracle.clover_field(U, dims, kappa, csw)
    x, _, _ = oracle.solve(U, F, kappa, b, tol=1e-14)
    lam = oracle.adjoint_solve(U, F, kappa, eta, tol=1e-14)
    G = oracle.link_grad(U, lam, x, kappa, csw)

    def L(Uh):
        Fh = oracle.clover_field(Uh, dims, kappa, csw)
        xh, _, _ = oracle.solve(Uh, Fh, kappa, b, tol=1e-14)
        return float(np.real(np.vdot(eta.reshape(-1), xh.reshape(-1))))

    for k in range(3):
        X = tangent(U, 360 + k)
        fd = fd_richardson(L, U, X, 1e-3)
        an = directional(G, X, U)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (k, fd, an)
    # the gradient with respect to b is lam (L is linear in b)
    db = synth.gaussian_source(dims, 370)
    fdb = float(np.real(np.vdot(eta.reshape(-1), oracle.solve(U, F, kappa, db, tol=1e-14)[0].reshape(-1))))
    assert abs(fdb - float(np.real(np.vdot(lam.reshape(-1), db.reshape(-1))))) < 1e-10 * abs(fdb)
