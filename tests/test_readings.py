"""The readings of the printed solver listings, decided on the CPU.

Algorithms 1 and 2 print alpha = <r~|q> and beta = (rho1/rho0)/(alpha/omega).
Read literally, alpha lacks the factor rho0 and beta is inverted.  On a small
even-odd system (dense D-hat_ee from the oracle) the textbook forms
alpha = rho0/<r~|q>, beta = (rho1/rho0)(alpha/omega) converge, and the literal
forms do not, which is why both the GPU solver and this repository read the
listings that way.
"""
import numpy as np

import oracle
import synth


def bicgstab(A, b, literal, tol=1e-10, maxit=400):
    # the iteration of Algorithm 2 on a dense matrix, either exactly as printed or
    # with the textbook alpha and beta
    x = np.zeros_like(b)
    r = b.copy()
    rt = r.copy()
    p = r.copy()
    rho0 = np.vdot(rt, r)
    nb = np.linalg.norm(b)
    for it in range(maxit):
        q = A @ p
        alpha = np.vdot(rt, q) if literal else rho0 / np.vdot(rt, q)
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) / nb < tol:
            return x, it, True
        t = A @ r
        omega = np.vdot(t, r) / np.vdot(t, t)
        x = x + omega * r
        r = r - omega * t
        if np.linalg.norm(r) / nb < tol:
            return x, it, True
        rho1 = np.vdot(rt, r)
        beta = (rho1 / rho0) / (alpha / omega) if literal else (rho1 / rho0) * (alpha / omega)
        rho0 = rho1
        p = r + beta * (p - omega * q)
        if not np.all(np.isfinite(x)):
            break
    return x, maxit, False


def test_textbook_forms_converge_literal_ones_do_not():
    dims = (4, 4, 4, 4)
    kappa = 0.13
    U = synth.random_links(dims, 0.3, 501)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    Finv = oracle.site_invert(F)
    b = synth.gaussian_source(dims, 502)
    even = (oracle.parity(dims) == 0).reshape(-1)
    idx = np.nonzero(np.repeat(even, 12))[0]
    n = idx.size
    A = np.empty((n, n), dtype=complex)
    e = np.zeros(b.size, dtype=complex)
    for j in range(n):
        e[:] = 0
        e[idx[j]] = 1
        A[:, j] = oracle.dhat_ee(U, Finv, kappa, e.reshape(b.shape)).reshape(-1)[idx]
    bh = oracle.bhat_e(U, Finv, kappa, b).reshape(-1)[idx]
    x, it, ok = bicgstab(A, bh, literal=False)
    assert ok and np.linalg.norm(A @ x - bh) / np.linalg.norm(bh) < 1e-9
    x_lit, it_lit, ok_lit = bicgstab(A, bh, literal=True)
    assert not ok_lit
