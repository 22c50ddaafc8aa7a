"""Seeded synthetic inputs for the Wilson-clover solver (gauge links and sources).

This module only draws random numbers and assembles input fields.  It holds
none of the operator's arithmetic: no hopping term, no clover term, no solver.
Both the FP64 oracle tests and the GPU path take their inputs from here.

Canonical layouts (complex128, C order), with lattice extents
``dims = (Lx, Ly, Lz, Lt)``:

* gauge links ``U[mu, t, z, y, x, i, j]`` for mu = x, y, z, t = 0..3;
  ``U[mu](n)`` is the 3x3 matrix on the link from n to n + mu-hat;
* spinors ``psi[t, z, y, x, alpha, a]`` with spin alpha = 0..3 and colour
  a = 0..2.

Random links follow the recipe U = exp(i * eps * H) with H a Gaussian
traceless Hermitian 3x3 matrix per link: A has independent N(0,1) real and
imaginary parts, H = (A + A^dagger)/2 - tr(.)/3.  Draws come from numpy's
PCG64 in canonical (mu, t, z, y, x, i, j, re/im) order.  The exponential of
the Hermitian matrix uses the closed Cayley-Hamilton form of Morningstar and
Peardon (Phys. Rev. D 69, 054501, 2004), which is exact up to rounding and
fast for many small matrices.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "expi_hermitian",
    "random_hermitian_traceless",
    "random_links",
    "random_links_torch",
    "unit_links",
    "haar_su3",
    "pure_gauge_links",
    "gauge_transform_links",
    "abelian_flux_links",
    "gaussian_source",
    "z2_source",
    "point_source",
    "shape_links",
    "shape_spinor",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def shape_links(dims):
    lx, ly, lz, lt = dims
    return (4, lt, lz, ly, lx, 3, 3)


def shape_spinor(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 4, 3)


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def random_hermitian_traceless(shape, g: np.random.Generator) -> np.ndarray:
    """Gaussian traceless Hermitian 3x3 matrices with leading ``shape``."""
    a = g.standard_normal(tuple(shape) + (3, 3, 2))
    a = a[..., 0] + 1j * a[..., 1]
    h = 0.5 * (a + _dag(a))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h[..., 0, 0] -= tr
    h[..., 1, 1] -= tr
    h[..., 2, 2] -= tr
    return h


def expi_hermitian(q: np.ndarray) -> np.ndarray:
    """exp(i Q) for traceless Hermitian 3x3 Q (batched over leading axes).

    Closed form exp(iQ) = f0 + f1 Q + f2 Q^2 (Morningstar-Peardon 2004): the
    coefficients follow from the two invariants c0 = det Q and c1 = tr Q^2 / 2.
    """
    q = np.asarray(q, dtype=np.complex128)
    q2 = q @ q
    c1 = 0.5 * np.trace(q2, axis1=-2, axis2=-1).real
    c0 = (np.trace(q2 @ q, axis1=-2, axis2=-1).real) / 3.0
    neg = c0 < 0
    c0a = np.abs(c0)
    c0max = 2.0 * np.power(np.maximum(c1, 0.0) / 3.0, 1.5)
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(c0max > 0, c0a / np.where(c0max > 0, c0max, 1.0), 0.0)
    theta = np.arccos(np.clip(ratio, -1.0, 1.0))
    u = np.sqrt(np.maximum(c1, 0.0) / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(np.maximum(c1, 0.0)) * np.sin(theta / 3.0)
    w2 = w * w
    u2 = u * u
    small = np.abs(w) < 0.05
    with np.errstate(invalid="ignore", divide="ignore"):
        xi0 = np.where(small,
                       1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)),
                       np.sin(w) / np.where(small, 1.0, w))
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    cw = np.cos(w)
    h0 = (u2 - w2) * e2iu + emiu * (8.0 * u2 * cw + 2j * u * (3.0 * u2 + w2) * xi0)
    h1 = 2.0 * u * e2iu - emiu * (2.0 * u * cw - 1j * (3.0 * u2 - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9.0 * u2 - w2
    zero = den == 0.0
    den = np.where(zero, 1.0, den)
    f0 = np.where(zero, 1.0, h0 / den)
    f1 = np.where(zero, 0.0, h1 / den)
    f2 = np.where(zero, 0.0, h2 / den)
    # the closed form was evaluated for |c0|; c0 -> -c0 maps f_j -> (-1)^j conj(f_j)
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    out = f1[..., None, None] * q + f2[..., None, None] * q2
    out[..., 0, 0] += f0
    out[..., 1, 1] += f0
    out[..., 2, 2] += f0
    return out


def random_links(dims, eps: float = 0.3, seed: int = 0, chunk_sites: int = 1 << 18) -> np.ndarray:
    """U_mu(n) = exp(i eps H), H Gaussian traceless Hermitian, canonical layout.

    Generated in chunks along (mu, t, z, y, x) so memory stays bounded; the
    PCG64 stream is consumed in the same order as one whole-array draw.
    """
    g = rng(seed)
    shp = shape_links(dims)
    out = np.empty(shp, dtype=np.complex128)
    flat = out.reshape(-1, 3, 3)
    nlinks = flat.shape[0]
    for s in range(0, nlinks, chunk_sites):
        e = min(nlinks, s + chunk_sites)
        h = random_hermitian_traceless((e - s,), g)
        flat[s:e] = expi_hermitian(eps * h)
    return out


def unit_links(dims) -> np.ndarray:
    out = np.zeros(shape_links(dims), dtype=np.complex128)
    out[..., 0, 0] = 1.0
    out[..., 1, 1] = 1.0
    out[..., 2, 2] = 1.0
    return out


def haar_su3(shape, g: np.random.Generator) -> np.ndarray:
    """Haar-random SU(3) matrices: QR of a complex Gaussian, phases fixed, det 1."""
    a = g.standard_normal(tuple(shape) + (3, 3, 2))
    a = a[..., 0] + 1j * a[..., 1]
    qm, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    qm = qm * ph[..., None, :]
    det = np.linalg.det(qm)
    qm = qm / np.power(det, 1.0 / 3.0)[..., None, None]
    return qm


def _shift(field, dims, mu, step):
    """field(n + step * mu-hat) for a site field laid out [t, z, y, x, ...]."""
    axis = 3 - mu
    return np.roll(field, -step, axis=axis)


def pure_gauge_links(omega: np.ndarray, dims) -> np.ndarray:
    """U_mu(n) = Omega(n) Omega(n + mu-hat)^dagger for a site field Omega[t,z,y,x,3,3]."""
    out = np.empty(shape_links(dims), dtype=np.complex128)
    for mu in range(4):
        out[mu] = omega @ _dag(_shift(omega, dims, mu, 1))
    return out


def gauge_transform_links(u: np.ndarray, omega: np.ndarray, dims) -> np.ndarray:
    """U^Omega_mu(n) = Omega(n) U_mu(n) Omega(n + mu-hat)^dagger."""
    out = np.empty_like(u)
    for mu in range(4):
        out[mu] = omega @ u[mu] @ _dag(_shift(omega, dims, mu, 1))
    return out


def abelian_flux_links(dims, k: int = 1, plane=(0, 1), charges=(1, 1, -2)) -> np.ndarray:
    """Diagonal U(1)^3 links carrying a constant flux through every (mu, nu) plaquette.

    Flux b = 2 pi k / (L_mu L_nu); colour c carries charge q_c.  Links:
    U_nu(n) = diag(exp(i q_c b n_mu)); U_mu(n) = 1 except on the last mu-slice,
    where U_mu(n) = diag(exp(-i q_c b L_mu n_nu)); every other link is 1.  Every
    counter-clockwise (mu, nu) plaquette then equals diag(exp(i q_c b)).
    """
    mu, nu = plane
    lx, ly, lz, lt = dims
    ext = [lx, ly, lz, lt]
    b = 2.0 * np.pi * k / (ext[mu] * ext[nu])
    q = np.asarray(charges, dtype=np.float64)
    u = unit_links(dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    coord = [x, y, z, t]
    nmu = coord[mu]
    nnu = coord[nu]
    for c in range(3):
        u[nu][..., c, c] = np.exp(1j * q[c] * b * nmu)
        ph = np.where(nmu == ext[mu] - 1, np.exp(-1j * q[c] * b * ext[mu] * nnu), 1.0)
        u[mu][..., c, c] = ph
    return u


def gaussian_source(dims, seed: int) -> np.ndarray:
    g = rng(seed)
    a = g.standard_normal(shape_spinor(dims) + (2,))
    return a[..., 0] + 1j * a[..., 1]


def z2_source(dims, seed: int) -> np.ndarray:
    """Real +-1 on every complex component (imaginary part 0)."""
    g = rng(seed)
    s = g.integers(0, 2, size=shape_spinor(dims)).astype(np.float64)
    return (2.0 * s - 1.0).astype(np.complex128)


def point_source(dims, alpha: int, a: int, site=(0, 0, 0, 0)) -> np.ndarray:
    out = np.zeros(shape_spinor(dims), dtype=np.complex128)
    x, y, z, t = site
    out[t, z, y, x, alpha, a] = 1.0
    return out


def _expi_hermitian_torch(q):
    """exp(i Q) for traceless Hermitian 3x3 Q in torch (any device), the same
    Cayley-Hamilton closed form as ``expi_hermitian``."""
    import torch

    q2 = q @ q
    c1 = 0.5 * torch.diagonal(q2, dim1=-2, dim2=-1).sum(-1).real
    c0 = torch.diagonal(q2 @ q, dim1=-2, dim2=-1).sum(-1).real / 3.0
    neg = c0 < 0
    c0a = c0.abs()
    c1p = torch.clamp(c1, min=0.0)
    c0max = 2.0 * (c1p / 3.0) ** 1.5
    ratio = torch.where(c0max > 0, c0a / torch.where(c0max > 0, c0max, torch.ones_like(c0max)),
                        torch.zeros_like(c0a))
    theta = torch.arccos(torch.clamp(ratio, -1.0, 1.0))
    u = torch.sqrt(c1p / 3.0) * torch.cos(theta / 3.0)
    w = torch.sqrt(c1p) * torch.sin(theta / 3.0)
    w2, u2 = w * w, u * u
    small = w.abs() < 0.05
    xi0 = torch.where(small, 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)),
                      torch.sin(w) / torch.where(small, torch.ones_like(w), w))
    e2iu = torch.exp(2j * u)
    emiu = torch.exp(-1j * u)
    cw = torch.cos(w)
    h0 = (u2 - w2) * e2iu + emiu * (8.0 * u2 * cw + 2j * u * (3.0 * u2 + w2) * xi0)
    h1 = 2.0 * u * e2iu - emiu * (2.0 * u * cw - 1j * (3.0 * u2 - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9.0 * u2 - w2
    zero = den == 0.0
    den = torch.where(zero, torch.ones_like(den), den)
    f0 = torch.where(zero, torch.ones_like(h0), h0 / den)
    f1 = torch.where(zero, torch.zeros_like(h1), h1 / den)
    f2 = torch.where(zero, torch.zeros_like(h2), h2 / den)
    f0 = torch.where(neg, f0.conj(), f0)
    f1 = torch.where(neg, -f1.conj(), f1)
    f2 = torch.where(neg, f2.conj(), f2)
    out = f1[..., None, None] * q + f2[..., None, None] * q2
    eye = torch.eye(3, dtype=q.dtype, device=q.device)
    return out + f0[..., None, None] * eye


def random_links_torch(dims, eps: float = 0.3, seed: int = 0, device="cuda", chunk_sites: int = 1 << 22):
    """``random_links`` with the exponential evaluated by torch on ``device``.

    The Gaussian draws are the same PCG64 stream in the same order as
    ``random_links``; the two results agree to rounding (~1e-15).  Returns a
    complex128 torch tensor (4, Lt, Lz, Ly, Lx, 3, 3) on ``device``.
    """
    import torch

    g = rng(seed)
    shp = shape_links(dims)
    out = torch.empty(shp, dtype=torch.complex128, device=device)
    flat = out.view(-1, 3, 3)
    nlinks = flat.shape[0]
    for s in range(0, nlinks, chunk_sites):
        e = min(nlinks, s + chunk_sites)
        h = torch.from_numpy(random_hermitian_traceless((e - s,), g)).to(device)
        flat[s:e] = _expi_hermitian_torch(eps * h)
    return out
