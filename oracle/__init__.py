"""FP64 CPU oracle for the Wilson-clover quark solver (arXiv:1709.08785).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may use this package; the GPU library never does.

The heavy loops live in ``oracle.c`` (plain C, FP64, OpenMP), loaded here with
ctypes.  Every function takes and returns numpy complex128 arrays in the
canonical layouts: links ``U[mu, t, z, y, x, 3, 3]`` and spinors
``psi[t, z, y, x, 4, 3]``; extents are ``dims = (Lx, Ly, Lz, Lt)``.

Functions and the passage each one follows:

* ``gamma``           Dirac matrices, Hermitian with g_t diagonal (Sec. II-A)
* ``hop``             hopping matrix H (Sec. II-A, eq. 4)
* ``clover_field``    clover term F(n), Sheikholeslami-Wohlert (Sec. II-A)
* ``apply_D``         D = F - kappa H (Sec. II-A, eq. 3)
* ``solve``           x = D^-1 b by plain BiCGStab on the full D, checked on
                      the true residual; ``dense_solve`` by LU for tiny lattices
* ``bhat_e``, ``dhat_ee``, ``x_o``  even-odd Schur pieces (Sec. II-B, eqs. 5-9);
                      ``clover_sites``, ``htilde_sites``, ``dhat_ee_sites``
                      F or F^-1, MULT and D-hat_ee at listed sites
* ``free_solve_fft``  D^-1 b for unit links by Fourier transform (eqs. 3-4
                      with U = 1 and F = 1)
* ``link_grad``       gradient of -Re<lam, D[U] x> with respect to the links
                      (the chain rule through eqs. 3-4 and the clover term)
* ``gamma5``, ``adjoint_solve``  D^-dagger = g5 D^-1 g5 (gamma5-hermiticity)
* ``fp32_storage``, ``fp16_storage``  what a spinor reads back as after storage
                      in single precision (Sec. III-A) or in the FP16 storage
                      format with a per-site scale (a reading: the paper's
                      method stores single and double precision only)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        lib.or_gamma.argtypes = [ctypes.c_int, P]
        lib.or_hop.argtypes = [P, P, P, P]
        lib.or_clover_field.argtypes = [P, P, D, D, P]
        lib.or_clover_leaves.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P]
        lib.or_site_apply.argtypes = [P, P, P, P]
        lib.or_site_invert.argtypes = [P, P, P]
        lib.or_site_invert.restype = ctypes.c_long
        lib.or_apply_D.argtypes = [P, P, P, D, P, P]
        lib.or_apply_D_sites.argtypes = [P, P, D, D, P, P, ctypes.c_long, P]
        lib.or_residual.argtypes = [P, P, D, D, P, P, P, P]
        lib.or_dhat_ee_sites.argtypes = [P, P, D, D, P, P, ctypes.c_long, P]
        lib.or_dhat_ee_sites.restype = ctypes.c_long
        lib.or_htilde_sites.argtypes = [P, P, D, D, P, P, ctypes.c_long, P]
        lib.or_htilde_sites.restype = ctypes.c_long
        lib.or_clover_sites.argtypes = [P, P, D, D, P, P, ctypes.c_long, ctypes.c_int, P]
        lib.or_clover_sites.restype = ctypes.c_long
        lib.or_bicgstab.argtypes = [P, P, P, D, P, P, D, ctypes.c_int, P, P]
        lib.or_bicgstab.restype = ctypes.c_int
        lib.or_link_grad.argtypes = [P, P, P, P, D, D, ctypes.c_int, P]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,)
    return d


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(n: int) -> None:
    _load().or_set_num_threads(int(n))


def dims_of_spinor(psi):
    lt, lz, ly, lx = psi.shape[:4]
    return (lx, ly, lz, lt)


def gamma(mu: int) -> np.ndarray:
    """g_mu, mu = 0..3 for x, y, z, t; mu = 4 gives g5 = g_x g_y g_z g_t."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().or_gamma(int(mu), _p(out))
    return out


def hop(U, psi) -> np.ndarray:
    """H psi, eq. (4), periodic boundaries."""
    dims = dims_of_spinor(psi)
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    L = _dims(dims)
    _load().or_hop(_p(L), _p(U), _p(psi), _p(out))
    return out


def clover_field(U, dims, kappa: float, csw: float) -> np.ndarray:
    """F(n) as 12x12 matrices, shape (Lt, Lz, Ly, Lx, 12, 12), index 3*alpha + a."""
    lx, ly, lz, lt = dims
    U = _c(U)
    F = np.empty((lt, lz, ly, lx, 12, 12), dtype=np.complex128)
    L = _dims(dims)
    _load().or_clover_field(_p(L), _p(U), float(kappa), float(csw), _p(F))
    return F


def clover_leaves(U, dims, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(n): sum of the four counter-clockwise plaquettes, shape (..., 3, 3)."""
    lx, ly, lz, lt = dims
    U = _c(U)
    Q = np.empty((lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    L = _dims(dims)
    _load().or_clover_leaves(_p(L), _p(U), int(mu), int(nu), _p(Q))
    return Q


def site_apply(M, psi) -> np.ndarray:
    dims = dims_of_spinor(psi)
    M, psi = _c(M), _c(psi)
    out = np.empty_like(psi)
    _load().or_site_apply(_p(_dims(dims)), _p(M), _p(psi), _p(out))
    return out


def site_invert(M) -> np.ndarray:
    lt, lz, ly, lx = M.shape[:4]
    M = _c(M)
    out = np.empty_like(M)
    bad = _load().or_site_invert(_p(_dims((lx, ly, lz, lt))), _p(M), _p(out))
    if bad:
        raise ArithmeticError("%d singular site matrices" % bad)
    return out


def apply_D(U, F, kappa: float, psi) -> np.ndarray:
    """D psi = F psi - kappa H psi, eq. (3)."""
    dims = dims_of_spinor(psi)
    U, F, psi = _c(U), _c(F), _c(psi)
    out = np.empty_like(psi)
    _load().or_apply_D(_p(_dims(dims)), _p(U), _p(F), float(kappa), _p(psi), _p(out))
    return out


def apply_D_sites(U, kappa: float, csw: float, psi, sites) -> np.ndarray:
    """(D psi)(n) for lexicographic site indices ``sites``; F(n) built on the fly."""
    dims = dims_of_spinor(psi)
    U, psi = _c(U), _c(psi)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.empty((s.size, 4, 3), dtype=np.complex128)
    _load().or_apply_D_sites(_p(_dims(dims)), _p(U), float(kappa), float(csw), _p(psi),
                             _p(s), ctypes.c_long(s.size), _p(out))
    return out


def residual(U, kappa: float, csw: float, b, x):
    """(||b - D x||, ||b||) over the whole lattice, F built on the fly."""
    dims = dims_of_spinor(b)
    U, b, x = _c(U), _c(b), _c(x)
    r2 = ctypes.c_double()
    b2 = ctypes.c_double()
    _load().or_residual(_p(_dims(dims)), _p(U), float(kappa), float(csw), _p(b), _p(x),
                        ctypes.byref(r2), ctypes.byref(b2))
    return float(np.sqrt(r2.value)), float(np.sqrt(b2.value))


def solve(U, F, kappa: float, b, tol: float = 1e-13, maxit: int = 20000, x0=None):
    """x = D^-1 b by plain BiCGStab on the full operator; returns (x, iters, true relres)."""
    dims = dims_of_spinor(b)
    U, F, b = _c(U), _c(F), _c(b)
    x = np.zeros_like(b) if x0 is None else _c(x0).copy()
    it = ctypes.c_int()
    rr = ctypes.c_double()
    st = _load().or_bicgstab(_p(_dims(dims)), _p(U), _p(F), float(kappa), _p(b), _p(x), float(tol),
                             int(maxit), ctypes.byref(it), ctypes.byref(rr))
    if st != 0:
        raise ArithmeticError("oracle BiCGStab did not converge (status %d, relres %.3e after %d)"
                              % (st, rr.value, it.value))
    return x, it.value, rr.value


def dense_matrix(U, F, kappa: float, dims) -> np.ndarray:
    """D as a dense (12V x 12V) matrix, columns from unit vectors (tiny lattices only)."""
    lx, ly, lz, lt = dims
    n = lx * ly * lz * lt * 12
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    ef = e.reshape(-1)
    for j in range(n):
        ef[:] = 0
        ef[j] = 1
        M[:, j] = apply_D(U, F, kappa, e).reshape(-1)
    return M


def dense_solve(U, F, kappa: float, b) -> np.ndarray:
    """x = D^-1 b by LU of the dense matrix (LAPACK through numpy)."""
    dims = dims_of_spinor(b)
    M = dense_matrix(U, F, kappa, dims)
    return np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)


# ---------------------------------------------------------------------------
# even-odd pieces (Sec. II-B, eqs. 5-9), built from the full-lattice routines
# ---------------------------------------------------------------------------

def parity(dims) -> np.ndarray:
    """(n_x + n_y + n_z + n_t) mod 2 laid out [t, z, y, x] (Sec. II-B)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return (x + y + z + t) & 1


def restrict(psi, par: int) -> np.ndarray:
    """Zero every site whose parity differs from ``par``."""
    m = parity(dims_of_spinor(psi)) == par
    return psi * m[..., None, None]


def htilde(U, Finv, psi, out_parity: int) -> np.ndarray:
    """H-tilde_{p,1-p} psi = F_pp^-1 H_{p,1-p} psi_{1-p}: MULT (Sec. II-B, eq. 9)."""
    h = hop(U, restrict(psi, 1 - out_parity))
    return restrict(site_apply(Finv, h), out_parity)


def dhat_ee(U, Finv, kappa: float, xe) -> np.ndarray:
    """D-hat_ee x_e = x_e - kappa^2 H-tilde_eo H-tilde_oe x_e (Sec. II-B, eq. 8, typo read as H_eo H_oe)."""
    xe = restrict(xe, 0)
    return xe - kappa * kappa * htilde(U, Finv, htilde(U, Finv, xe, 1), 0)


def clover_sites(U, kappa: float, csw: float, psi, sites, inverse: bool = False) -> np.ndarray:
    """F(n) psi(n), or F(n)^-1 psi(n), at lexicographic sites ``sites``
    (Sec. II-A; Sec. II-B for the inverse), F built from the links on the fly."""
    dims = dims_of_spinor(psi)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    U, psi = _c(U), _c(psi)
    out = np.empty((s.size, 4, 3), dtype=np.complex128)
    bad = _load().or_clover_sites(_p(_dims(dims)), _p(U), float(kappa), float(csw), _p(psi),
                                  _p(s), ctypes.c_long(s.size), int(bool(inverse)), _p(out))
    if bad:
        raise ArithmeticError("%d singular clover matrices" % bad)
    return out


def htilde_sites(U, kappa: float, csw: float, psi, sites) -> np.ndarray:
    """MULT F(n)^-1 (H psi)(n) at lexicographic sites ``sites`` (Sec. II-B, eq. 9);
    only the neighbours of each site, of the other parity, are read.  Clover
    blocks are built and inverted on the fly."""
    dims = dims_of_spinor(psi)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    U, psi = _c(U), _c(psi)
    out = np.empty((s.size, 4, 3), dtype=np.complex128)
    bad = _load().or_htilde_sites(_p(_dims(dims)), _p(U), float(kappa), float(csw), _p(psi),
                                  _p(s), ctypes.c_long(s.size), _p(out))
    if bad:
        raise ArithmeticError("%d singular clover matrices" % bad)
    return out


def dhat_ee_sites(U, kappa: float, csw: float, xe, sites) -> np.ndarray:
    """(D-hat_ee xe)(n) at even lexicographic sites ``sites`` (Sec. II-B, eq. 8,
    same reading as ``dhat_ee``); clover blocks built and inverted on the fly,
    so it serves lattices whose whole clover field would not fit."""
    dims = dims_of_spinor(xe)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    par = parity(dims).reshape(-1)[s]
    if np.any(par != 0):
        raise ValueError("dhat_ee_sites takes even sites only")
    U, xe = _c(U), _c(xe)
    out = np.empty((s.size, 4, 3), dtype=np.complex128)
    bad = _load().or_dhat_ee_sites(_p(_dims(dims)), _p(U), float(kappa), float(csw), _p(xe),
                                   _p(s), ctypes.c_long(s.size), _p(out))
    if bad:
        raise ArithmeticError("%d singular clover matrices" % bad)
    return out


def bhat_e(U, Finv, kappa: float, b) -> np.ndarray:
    """b-hat_e = F_ee^-1 b_e + kappa H-tilde_eo F_oo^-1 b_o (Sec. II-B, eq. 6)."""
    fb = site_apply(Finv, b)
    return restrict(fb, 0) + kappa * htilde(U, Finv, restrict(fb, 1), 0)


def x_o(U, Finv, kappa: float, b, xe) -> np.ndarray:
    """x_o = F_oo^-1 b_o + kappa H-tilde_oe x_e (Sec. II-B, eq. 7)."""
    return restrict(site_apply(Finv, b), 1) + kappa * htilde(U, Finv, restrict(xe, 0), 1)


# ---------------------------------------------------------------------------
# unit links: solve by Fourier transform
# ---------------------------------------------------------------------------

def free_momentum_operator(dims, kappa: float):
    """D(p) for unit links as (Lt, Lz, Ly, Lx, 4, 4) spin matrices.

    With U = 1 and F = 1, a plane wave e^{i p.n} u is an eigenvector of H with
    H -> sum_mu [(1 - g_mu) e^{i p_mu} + (1 + g_mu) e^{-i p_mu}]
       = sum_mu [2 cos p_mu - 2 i g_mu sin p_mu].
    """
    lx, ly, lz, lt = dims
    ps = [2 * np.pi * np.arange(n) / n for n in (lx, ly, lz, lt)]
    pt, pz, py, px = np.meshgrid(ps[3], ps[2], ps[1], ps[0], indexing="ij")
    p = [px, py, pz, pt]
    eye = np.eye(4, dtype=np.complex128)
    D = np.zeros((lt, lz, ly, lx, 4, 4), dtype=np.complex128)
    D += eye
    for mu in range(4):
        g = gamma(mu)
        D -= kappa * (2 * np.cos(p[mu])[..., None, None] * eye
                      - 2j * np.sin(p[mu])[..., None, None] * g)
    return D


def free_solve_fft(b, kappa: float) -> np.ndarray:
    """x = D^-1 b for U = 1 (so F = 1) by diagonalising D in momentum space."""
    dims = dims_of_spinor(b)
    Dp = free_momentum_operator(dims, kappa)
    bt = np.fft.fftn(b, axes=(0, 1, 2, 3))
    xt = np.linalg.solve(Dp, bt)          # colour index acts as 3 right-hand sides
    return np.fft.ifftn(xt, axes=(0, 1, 2, 3))


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def gamma5(psi) -> np.ndarray:
    """g5 psi with g5 = g_x g_y g_z g_t."""
    return np.einsum("ab,...bc->...ac", gamma(4), psi)


def adjoint_solve(U, F, kappa: float, eta, tol: float = 1e-13):
    """lam = D^-dagger eta = g5 D^-1 g5 eta (D is gamma5-Hermitian)."""
    y, _, _ = solve(U, F, kappa, gamma5(eta), tol=tol)
    return gamma5(y)


def link_grad(U, lam, x, kappa: float, csw: float, include_clover: bool = True) -> np.ndarray:
    """G with dg = Re sum conj(G) dU for g(U) = -Re<lam, D[U] x> (lam, x fixed).

    At lam = D^-dagger eta, x = D^-1 b it is the link gradient of
    L = Re<eta, D^-1 b> in torch's complex convention (dL/dRe U + i dL/dIm U).
    """
    dims = dims_of_spinor(x)
    U, lam, x = _c(U), _c(lam), _c(x)
    G = np.zeros_like(U)
    _load().or_link_grad(_p(_dims(dims)), _p(U), _p(lam), _p(x), float(kappa), float(csw),
                         int(bool(include_clover)), _p(G))
    return G


# ---------------------------------------------------------------------------
# storage formats of the low-precision copies
# ---------------------------------------------------------------------------

def fp32_storage(psi) -> np.ndarray:
    """psi after a round trip through single precision: every real rounded to
    the nearest FP32, ties to even (the SP copies of Sec. III-A)."""
    return np.asarray(psi, dtype=np.complex128).astype(np.complex64).astype(np.complex128)


def fp16_storage(psi) -> np.ndarray:
    """psi after a round trip through the FP16 storage format (a reading; the
    paper stores single and double precision only).

    Encoding of one site, all steps in FP32 with round-to-nearest-even:
    the 24 reals are rounded to FP32; the scale s is the largest of their
    magnitudes; each real is multiplied by r = 1/s (r = 0 when s = 0) and
    rounded to the nearest FP16.  Decoding multiplies each FP16 value, read as
    FP32, by s.  The encoded values lie in [-1, 1]; small ones may become FP16
    subnormals, which are kept.
    """
    v = np.asarray(psi, dtype=np.complex128).astype(np.complex64)
    re = np.stack([v.real, v.imag], axis=-1).astype(np.float32)      # [..., 4, 3, 2]
    sites = re.reshape(re.shape[:-3] + (24,))
    s = np.abs(sites).max(axis=-1, keepdims=True).astype(np.float32)
    with np.errstate(divide="ignore"):
        r = np.where(s > 0, np.float32(1.0) / s, np.float32(0.0)).astype(np.float32)
    h = (sites * r).astype(np.float32).astype(np.float16)
    dec = (h.astype(np.float32) * s).astype(np.float32).reshape(re.shape)
    return (dec[..., 0].astype(np.float64) + 1j * dec[..., 1].astype(np.float64))
