"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

None of these tests compares the oracle with itself: each expected value is a
closed form worked out by hand (free-field momentum-space operator, constant
abelian flux), a symmetry of the operator (gamma5-hermiticity, gauge and
translation covariance), or an independent library route (dense LU).  The
numbers the paper prints (Tables 1 and 2, the byte model of Sec. IV-B) are
fixtures under tests/golden/, checked in test_paper_tables.py.
"""
import numpy as np
import pytest

import oracle
import synth

# ---------------------------------------------------------------------------
# Dirac representation written out by hand from the Pauli matrices:
#   g_k = [[0, -i s_k], [i s_k, 0]],  g_t = diag(1, 1, -1, -1)
# ---------------------------------------------------------------------------
I_ = 1j
G_HAND = [
    np.array([[0, 0, 0, -I_], [0, 0, -I_, 0], [0, I_, 0, 0], [I_, 0, 0, 0]]),
    np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=complex),
    np.array([[0, 0, -I_, 0], [0, 0, 0, I_], [I_, 0, 0, 0], [0, -I_, 0, 0]]),
    np.diag([1, 1, -1, -1]).astype(complex),
]
G5_HAND = np.array([[0, 0, -1, 0], [0, 0, 0, -1], [-1, 0, 0, 0], [0, -1, 0, 0]], dtype=complex)

# g_mu g_nu for mu < nu, also by hand: spatial pairs are block-diagonal
# diag(s_k s_l, s_k s_l); pairs with t are [[0, i s_k], [i s_k, 0]].
_SX = np.array([[0, 1], [1, 0]], dtype=complex)
_SY = np.array([[0, -1j], [1j, 0]])
_SZ = np.array([[1, 0], [0, -1]], dtype=complex)
_Z2 = np.zeros((2, 2), dtype=complex)


def _bd(a):
    return np.block([[a, _Z2], [_Z2, a]])


def _off(a):
    return np.block([[_Z2, a], [a, _Z2]])


GG_HAND = {
    (0, 1): _bd(1j * _SZ),            # s_x s_y = i s_z
    (0, 2): _bd(-1j * _SY),           # s_x s_z = -i s_y
    (1, 2): _bd(1j * _SX),            # s_y s_z = i s_x
    (0, 3): _off(1j * _SX),
    (1, 3): _off(1j * _SY),
    (2, 3): _off(1j * _SZ),
}


def g5_apply(psi):
    return np.einsum("ab,...bc->...ac", G5_HAND, psi)


def vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def rel(a, b):
    return np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1))


# ---------------------------------------------------------------------------
# gamma matrices (Sec. II-A: Hermitian, g_t diagonal)
# ---------------------------------------------------------------------------

def test_gamma_matches_hand_dirac_representation():
    for mu in range(4):
        assert np.array_equal(oracle.gamma(mu), G_HAND[mu])
    assert np.allclose(oracle.gamma(4), G5_HAND, atol=0, rtol=0)


def test_gamma_clifford_hermitian_tdiag():
    g = [oracle.gamma(m) for m in range(5)]
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2 * (m == n) * np.eye(4))
        assert np.allclose(g[4] @ g[m] + g[m] @ g[4], 0)
    assert np.allclose(g[3], np.diag(np.diag(g[3])))
    assert np.allclose(g[4] @ g[4], np.eye(4))


# ---------------------------------------------------------------------------
# free field (U = 1): plane waves are eigenvectors, closed-form D(p)
# ---------------------------------------------------------------------------

DIMS_NC = (4, 6, 8, 10)   # non-cubic: an axis swap changes the answer


def _plane_wave(dims, k, u):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    p = [2 * np.pi * k[i] / dims[i] for i in range(4)]
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * u[None, None, None, None], p


def _Dp_hand(p, kappa):
    # D(p) = (1 - 2 kappa sum cos p) + 2 i kappa sum g_mu sin p_mu
    m = (1 - 2 * kappa * sum(np.cos(q) for q in p)) * np.eye(4, dtype=complex)
    for mu in range(4):
        m = m + 2j * kappa * np.sin(p[mu]) * G_HAND[mu]
    return m


@pytest.mark.parametrize("k", [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
                               (1, 2, 3, 4), (3, 5, 7, 9), (2, 3, 4, 5)])
def test_free_field_plane_wave(k):
    dims = DIMS_NC
    kappa = 0.13
    g = synth.rng(7)
    u = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
    psi, p = _plane_wave(dims, k, u)
    U = synth.unit_links(dims)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    out = oracle.apply_D(U, F, kappa, psi)
    expect = np.einsum("ab,...bc->...ac", _Dp_hand(p, kappa), psi)
    assert rel(out, expect) < 1e-14


def test_free_field_eigenvalues_closed_form():
    # eigenvalues 1 - 2k sum cos p +- 2 i k sqrt(sum sin^2 p), each 6-fold
    dims = DIMS_NC
    kappa = 0.12
    Dp = oracle.free_momentum_operator(dims, kappa)
    lx, ly, lz, lt = dims
    for (t, z, y, x) in [(0, 0, 0, 0), (1, 2, 3, 1), (9, 7, 5, 3), (5, 4, 3, 2)]:
        p = [2 * np.pi * x / lx, 2 * np.pi * y / ly, 2 * np.pi * z / lz, 2 * np.pi * t / lt]
        a = 1 - 2 * kappa * sum(np.cos(q) for q in p)
        s = 2 * kappa * np.sqrt(sum(np.sin(q) ** 2 for q in p))
        ev = np.linalg.eigvals(Dp[t, z, y, x])
        ev = ev[np.argsort(ev.imag)]
        expect = np.array([a - 1j * s, a - 1j * s, a + 1j * s, a + 1j * s])
        assert np.allclose(ev, expect, atol=1e-14)


def test_free_field_dhat_even_plane_wave():
    # D-hat_ee on an even-restricted plane wave = (1 - kappa^2 h(p)^2), with
    # h(p) = sum_mu [2 cos p_mu - 2 i g_mu sin p_mu]  (i.e. lambda (2 - lambda))
    dims = DIMS_NC
    kappa = 0.13
    U = synth.unit_links(dims)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    Finv = oracle.site_invert(F)
    g = synth.rng(3)
    u = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
    for k in [(1, 2, 3, 4), (0, 1, 0, 3), (2, 0, 5, 1)]:
        psi, p = _plane_wave(dims, k, u)
        pe = oracle.restrict(psi, 0)
        h = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * np.sin(p[m]) * G_HAND[m] for m in range(4))
        M = np.eye(4) - kappa ** 2 * h @ h
        out = oracle.dhat_ee(U, Finv, kappa, pe)
        expect = oracle.restrict(np.einsum("ab,...bc->...ac", M, psi), 0)
        assert rel(out, expect) < 1e-14
        # the eigenvalue relation lambda (2 - lambda) with lambda of D(p)
        lam = np.linalg.eigvals(_Dp_hand(p, kappa))
        ev = np.linalg.eigvals(M)
        mu2 = lam * (2 - lam)
        assert np.allclose(ev[np.argsort(ev.imag)], mu2[np.argsort(mu2.imag)], atol=1e-13)


def test_free_solve_fft_solves_D():
    dims = (4, 4, 6, 6)
    kappa = 0.12
    U = synth.unit_links(dims)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    b = synth.gaussian_source(dims, 11)
    x = oracle.free_solve_fft(b, kappa)
    assert rel(oracle.apply_D(U, F, kappa, x), b) < 1e-13


# ---------------------------------------------------------------------------
# clover term
# ---------------------------------------------------------------------------

def test_clover_unit_links_is_identity():
    dims = (4, 4, 4, 6)
    F = oracle.clover_field(synth.unit_links(dims), dims, 0.135, 1.0)
    assert np.array_equal(F, np.broadcast_to(np.eye(12), F.shape))


def test_clover_pure_gauge_is_identity():
    dims = (4, 4, 4, 6)
    om = synth.haar_su3((6, 4, 4, 4), synth.rng(5))
    U = synth.pure_gauge_links(om, dims)
    F = oracle.clover_field(U, dims, 0.135, 1.0)
    assert np.abs(F - np.eye(12)).max() < 1e-14


@pytest.mark.parametrize("plane", [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3)])
def test_clover_abelian_flux_closed_form(plane):
    # every (mu,nu) plaquette = diag(e^{i q_c b}) -> Fhat = diag(i sin q_c b);
    # F = 1 - kappa csw (g_mu g_nu) (x) diag(i sin q_c b); no trace subtraction
    dims = (4, 6, 8, 6)
    kappa, csw, k = 0.13, 1.0, 5
    q = np.array([1.0, 1.0, -2.0])
    U = synth.abelian_flux_links(dims, k=k, plane=plane, charges=q)
    ext = list(dims)
    b = 2 * np.pi * k / (ext[plane[0]] * ext[plane[1]])
    F = oracle.clover_field(U, dims, kappa, csw)
    expect = np.eye(12, dtype=complex) - kappa * csw * np.kron(GG_HAND[plane], np.diag(1j * np.sin(q * b)))
    assert np.abs(F - expect).max() < 1e-14
    # the traceless variant would differ by i (sum_c sin q_c b)/3 on the colour diagonal
    assert abs(np.sin(q * b).sum()) > 0.1
    # and F^-1 matches the inverse of the closed form
    Finv = oracle.site_invert(F)
    assert np.abs(Finv - np.linalg.inv(expect)).max() < 1e-14


def test_clover_leaves_orientation():
    # Q_{nu mu} = Q_{mu nu}^dagger for random links
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 0.3, 21)
    for mu, nu in [(0, 1), (1, 3), (2, 3)]:
        a = oracle.clover_leaves(U, dims, mu, nu)
        b = oracle.clover_leaves(U, dims, nu, mu)
        assert np.abs(a - np.conj(np.swapaxes(b, -1, -2))).max() < 1e-14


def test_clover_hermitian_chiral_blocks_and_bound():
    dims = (4, 4, 4, 6)
    kappa, csw = 0.1355, 1.0
    U = synth.random_links(dims, 0.3, 31)
    F = oracle.clover_field(U, dims, kappa, csw).reshape(-1, 12, 12)
    assert np.abs(F - np.conj(np.swapaxes(F, -1, -2))).max() < 1e-15
    g5 = np.kron(G5_HAND, np.eye(3))
    assert np.abs(F @ g5 - g5 @ F).max() < 1e-15
    # ||F - 1|| <= 6 kappa csw, so F is positive definite
    ev = np.linalg.eigvalsh(F)
    assert ev.min() > 1 - 6 * kappa * csw and ev.max() < 1 + 6 * kappa * csw
    Fi = oracle.site_invert(F.reshape(6, 4, 4, 4, 12, 12)).reshape(-1, 12, 12)
    assert np.abs(F @ Fi - np.eye(12)).max() < 1e-14


# ---------------------------------------------------------------------------
# symmetries with random links
# ---------------------------------------------------------------------------

def test_gamma5_hermiticity():
    dims = (4, 6, 4, 8)
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 41)
    F = oracle.clover_field(U, dims, kappa, csw)
    x = synth.gaussian_source(dims, 42)
    y = synth.gaussian_source(dims, 43)
    lhs = vdot(y, oracle.apply_D(U, F, kappa, x))
    rhs = vdot(g5_apply(oracle.apply_D(U, F, kappa, g5_apply(y))), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14


def test_gauge_covariance():
    dims = (4, 4, 6, 4)
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 51)
    om = synth.haar_su3((4, 6, 4, 4), synth.rng(52))
    Ug = synth.gauge_transform_links(U, om, dims)
    F = oracle.clover_field(U, dims, kappa, csw)
    Fg = oracle.clover_field(Ug, dims, kappa, csw)
    # F[U^Om] = Om F Om^dagger (colour part of each 12x12 block)
    O12 = np.einsum("ab,...ij->...aibj", np.eye(4), om).reshape(om.shape[:4] + (12, 12))
    assert np.abs(Fg - O12 @ F @ np.conj(np.swapaxes(O12, -1, -2))).max() < 1e-14
    psi = synth.gaussian_source(dims, 53)
    om_psi = np.einsum("...ij,...aj->...ai", om, psi)
    lhs = oracle.apply_D(Ug, Fg, kappa, om_psi)
    rhs = np.einsum("...ij,...aj->...ai", om, oracle.apply_D(U, F, kappa, psi))
    assert rel(lhs, rhs) < 1e-14


@pytest.mark.parametrize("shift", [(1, 0, 0, 0), (1, 1, 0, 0), (0, 0, 0, 1), (0, 3, 1, 5)])
def test_translation_covariance(shift):
    dims = (4, 6, 4, 8)
    kappa, csw = 0.12, 1.0
    U = synth.random_links(dims, 0.3, 61)
    psi = synth.gaussian_source(dims, 62)
    sx, sy, sz, st = shift
    axes_site = (0, 1, 2, 3)           # t, z, y, x for spinors

    def sh_spin(a):
        return np.roll(a, (st, sz, sy, sx), axis=axes_site)

    def sh_link(a):
        return np.roll(a, (st, sz, sy, sx), axis=(1, 2, 3, 4))

    F = oracle.clover_field(U, dims, kappa, csw)
    Us = sh_link(U)
    Fs = oracle.clover_field(Us, dims, kappa, csw)
    assert np.abs(Fs - sh_spin(F)).max() < 1e-15
    out = oracle.apply_D(Us, Fs, kappa, sh_spin(psi))
    assert rel(out, sh_spin(oracle.apply_D(U, F, kappa, psi))) < 1e-15


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,kappa", [((2, 2, 2, 2), 0.135), ((4, 4, 4, 4), 0.1355), ((4, 4, 4, 4), 0.12)])
def test_bicgstab_matches_dense_lu(dims, kappa):
    U = synth.random_links(dims, 0.3, 71)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    b = synth.gaussian_source(dims, 72)
    x_lu = oracle.dense_solve(U, F, kappa, b)
    x, it, rr = oracle.solve(U, F, kappa, b, tol=1e-14)
    assert rr < 1e-14
    assert rel(x, x_lu) < 1e-12
    r, bn = oracle.residual(U, kappa, 1.0, b, x_lu)
    assert r / bn < 1e-13


def test_even_odd_reconstruction_dense():
    # x_e from D-hat_ee x_e = b-hat_e (dense LU on the even sites), x_o from eq. 7:
    # the pair solves D x = b (eqs. 5-9 with the H_eo H_oe reading of eq. 8)
    dims = (4, 4, 4, 4)
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 81)
    F = oracle.clover_field(U, dims, kappa, csw)
    Finv = oracle.site_invert(F)
    b = synth.gaussian_source(dims, 82)
    even = (oracle.parity(dims) == 0).reshape(-1)
    idx = np.nonzero(np.repeat(even, 12))[0]
    n = idx.size
    M = np.empty((n, n), dtype=complex)
    e = np.zeros(b.size, dtype=complex)
    for j in range(n):
        e[:] = 0
        e[idx[j]] = 1
        M[:, j] = oracle.dhat_ee(U, Finv, kappa, e.reshape(b.shape)).reshape(-1)[idx]
    bh = oracle.bhat_e(U, Finv, kappa, b).reshape(-1)[idx]
    xe = np.zeros(b.size, dtype=complex)
    xe[idx] = np.linalg.solve(M, bh)
    xe = xe.reshape(b.shape)
    x = xe + oracle.x_o(U, Finv, kappa, b, xe)
    assert rel(oracle.apply_D(U, F, kappa, x), b) < 1e-13
    # the literal eq. 8 (H_eo H_eo) is not even defined: H_eo of an even-only
    # vector is zero, so it would give D-hat = 1, which does not solve D x = b
    x_lit = oracle.restrict(oracle.bhat_e(U, Finv, kappa, b), 0)
    x_lit = x_lit + oracle.x_o(U, Finv, kappa, b, x_lit)
    assert rel(oracle.apply_D(U, F, kappa, x_lit), b) > 1e-3


def test_schur_complement_gamma5_hermitian():
    # S_ee = F_ee D-hat_ee is gamma5-Hermitian (D-hat itself is not)
    dims = (4, 4, 4, 4)
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 91)
    F = oracle.clover_field(U, dims, kappa, csw)
    Finv = oracle.site_invert(F)
    x = oracle.restrict(synth.gaussian_source(dims, 92), 0)
    y = oracle.restrict(synth.gaussian_source(dims, 93), 0)

    def S(v):
        return oracle.site_apply(F, oracle.dhat_ee(U, Finv, kappa, v))

    lhs = vdot(y, S(x))
    rhs = vdot(g5_apply(S(g5_apply(y))), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14


def test_pure_gauge_fft_solve_and_residual():
    # D[U] = Om D_free Om^dagger for U_mu(n) = Om(n) Om(n+mu)^dagger
    dims = (4, 6, 4, 8)
    kappa = 0.12
    om = synth.haar_su3((8, 4, 6, 4), synth.rng(101))
    U = synth.pure_gauge_links(om, dims)
    b = synth.gaussian_source(dims, 102)
    omd_b = np.einsum("...ji,...aj->...ai", np.conj(om), b)
    x = np.einsum("...ij,...aj->...ai", om, oracle.free_solve_fft(omd_b, kappa))
    r, bn = oracle.residual(U, kappa, 1.0, b, x)
    assert r / bn < 1e-13
    F = oracle.clover_field(U, dims, kappa, 1.0)
    xs, it, rr = oracle.solve(U, F, kappa, b, tol=1e-13)
    assert rel(xs, x) < 1e-12


# ---------------------------------------------------------------------------
# the true residual ||b - D x|| (used to judge every full-size solve), pinned
# from both sides: exact values, not only "small for a solution"
# ---------------------------------------------------------------------------

def test_residual_of_zero_is_norm_b():
    # x = 0 leaves r = b: both returned norms equal ||b|| (numpy's norm)
    dims = (4, 4, 4, 6)
    U = synth.random_links(dims, 0.3, 111)
    b = synth.gaussian_source(dims, 112)
    r, bn = oracle.residual(U, 0.13, 1.0, b, np.zeros_like(b))
    nb = np.linalg.norm(b.reshape(-1))
    assert abs(r - nb) <= 1e-14 * nb and abs(bn - nb) <= 1e-14 * nb


def test_residual_free_field_plane_waves_closed_form():
    # unit links (F = 1): x = e^{ipn} u, b = e^{ipn} w gives b - D x = e^{ipn} (w - D(p) u),
    # so ||b - D x||^2 = V ||w - D(p) u||^2 with D(p) built from the hand-typed gammas.
    # u and w are complex, so a residual that drops imaginary parts is caught.
    dims = DIMS_NC
    kappa = 0.13
    g = synth.rng(113)
    U = synth.unit_links(dims)
    V = int(np.prod(dims))
    for k in [(1, 2, 3, 4), (0, 1, 0, 3), (3, 5, 7, 9)]:
        u = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        w = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        x, p = _plane_wave(dims, k, u)
        b, _ = _plane_wave(dims, k, w)
        expect = np.sqrt(V) * np.linalg.norm(w - _Dp_hand(p, kappa) @ u)
        r, bn = oracle.residual(U, kappa, 1.0, b, x)
        assert abs(r - expect) <= 1e-13 * expect
        assert abs(bn - np.sqrt(V) * np.linalg.norm(w)) <= 1e-13 * bn


def test_residual_of_a_non_solution_matches_apply_D():
    # random links with the clover term on, random x that solves nothing: the
    # residual equals ||b - D x|| from the pinned whole-lattice operator
    dims = (4, 6, 4, 4)
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 114)
    F = oracle.clover_field(U, dims, kappa, csw)
    b = synth.gaussian_source(dims, 115)
    x = synth.gaussian_source(dims, 116)
    expect = np.linalg.norm((b - oracle.apply_D(U, F, kappa, x)).reshape(-1))
    r, bn = oracle.residual(U, kappa, csw, b, x)
    assert abs(r - expect) <= 1e-14 * expect
    assert abs(bn - np.linalg.norm(b.reshape(-1))) <= 1e-14 * bn


def test_special_cases_kappa0_csw0():
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 0.3, 111)
    b = synth.gaussian_source(dims, 112)
    F0 = oracle.clover_field(U, dims, 0.0, 1.0)
    assert np.array_equal(oracle.apply_D(U, F0, 0.0, b), b)
    Fw = oracle.clover_field(U, dims, 0.13, 0.0)
    assert np.array_equal(Fw, np.broadcast_to(np.eye(12), Fw.shape))
    assert rel(oracle.apply_D(U, Fw, 0.13, b), b - 0.13 * oracle.hop(U, b)) < 1e-15


def test_apply_D_sites_matches_whole_lattice():
    dims = (4, 6, 4, 8)
    kappa, csw = 0.135, 1.0
    U = synth.random_links(dims, 0.3, 121)
    F = oracle.clover_field(U, dims, kappa, csw)
    psi = synth.gaussian_source(dims, 122)
    full = oracle.apply_D(U, F, kappa, psi).reshape(-1, 4, 3)
    sites = [0, 1, 5, 17, 100, 767]
    part = oracle.apply_D_sites(U, kappa, csw, psi, sites)
    assert np.abs(part - full[sites]).max() < 1e-14


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (6, 4, 2, 8)])
def test_clover_sites_matches_whole_lattice(dims):
    # F and F^-1 applied site by site against the whole-lattice field and its
    # inverse (F pinned by the abelian-flux closed form and the symmetries)
    kappa, csw = 0.1355, 1.0
    U = synth.random_links(dims, 0.3, 128)
    F = oracle.clover_field(U, dims, kappa, csw)
    psi = synth.gaussian_source(dims, 129)
    sites = np.arange(int(np.prod(dims)))[::-1]
    for inverse, M in ((False, F), (True, oracle.site_invert(F))):
        full = oracle.site_apply(M, psi).reshape(-1, 4, 3)
        part = oracle.clover_sites(U, kappa, csw, psi, sites, inverse)
        assert np.abs(part - full[sites]).max() < 1e-13 * np.abs(full).max(), inverse


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (6, 4, 2, 8)])
def test_htilde_sites_matches_whole_lattice(dims):
    # site-by-site MULT against the whole-lattice one, both output parities
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 126)
    Finv = oracle.site_invert(oracle.clover_field(U, dims, kappa, csw))
    psi = synth.gaussian_source(dims, 127)
    par = oracle.parity(dims).reshape(-1)
    for p in (0, 1):
        full = oracle.htilde(U, Finv, psi, p).reshape(-1, 4, 3)
        sites = np.flatnonzero(par == p)[::-1]
        part = oracle.htilde_sites(U, kappa, csw, oracle.restrict(psi, 1 - p), sites)
        assert np.abs(part - full[sites]).max() < 1e-13 * np.abs(full).max(), p
        # the sites' own parity is not read
        part = oracle.htilde_sites(U, kappa, csw, psi, sites)
        assert np.abs(part - full[sites]).max() < 1e-13 * np.abs(full).max(), p


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (6, 4, 2, 8)])
def test_dhat_ee_sites_matches_whole_lattice(dims):
    # the site-by-site D-hat_ee against the whole-lattice one (pinned by the
    # free-field eigenvalues and the even-odd reconstruction) at every even site
    kappa, csw = 0.13, 1.0
    U = synth.random_links(dims, 0.3, 123)
    Finv = oracle.site_invert(oracle.clover_field(U, dims, kappa, csw))
    xe = oracle.restrict(synth.gaussian_source(dims, 124), 0)
    full = oracle.dhat_ee(U, Finv, kappa, xe).reshape(-1, 4, 3)
    even = np.flatnonzero(oracle.parity(dims).reshape(-1) == 0)
    part = oracle.dhat_ee_sites(U, kappa, csw, xe, even[::-1])
    assert np.abs(part - full[even[::-1]]).max() < 1e-13 * np.abs(full).max()
    # odd sites of the input are not read; odd output sites are refused
    noisy = xe + oracle.restrict(synth.gaussian_source(dims, 125), 1)
    assert np.abs(oracle.dhat_ee_sites(U, kappa, csw, noisy, even) - full[even]).max() < 1e-13 * np.abs(full).max()
    with pytest.raises(ValueError):
        oracle.dhat_ee_sites(U, kappa, csw, xe, [int(np.flatnonzero(oracle.parity(dims).reshape(-1))[0])])


# ---------------------------------------------------------------------------
# storage formats: single precision (Sec. III-A) and the FP16 format with a
# per-site scale (a reading), pinned by rounding facts worked out by hand
# ---------------------------------------------------------------------------

def _site(vals):
    """One-site 2x2x2x2 spinor field whose site 0 holds the given reals
    (re, im interleaved, spin-major then colour) and every other site zero."""
    psi = np.zeros((2, 2, 2, 2, 4, 3), dtype=complex)
    v = np.zeros(24)
    v[:len(vals)] = vals
    psi[0, 0, 0, 0] = (v[0::2] + 1j * v[1::2]).reshape(4, 3)
    return psi


def _reals(psi):
    s = psi[0, 0, 0, 0].reshape(12)
    return np.stack([s.real, s.imag], axis=-1).reshape(24)


def test_fp32_storage_rounds_to_nearest_even():
    one = 1.0
    # 1 + 2^-24 lies halfway between 1 and 1 + 2^-23: ties to even gives 1;
    # 1 + 3 * 2^-24 lies halfway between 1 + 2^-23 and 1 + 2^-22: gives 1 + 2^-22
    got = _reals(oracle.fp32_storage(_site([one + 2 ** -24, one + 3 * 2 ** -24, 1.0 / 3.0])))
    assert got[0] == 1.0 and got[1] == 1.0 + 2 ** -22
    assert abs(got[2] - 1.0 / 3.0) <= 2 ** -26 and got[2] != 1.0 / 3.0


def test_fp16_storage_exact_cases():
    # scale a power of two and values k/1024 * s: every step is exact
    vals = [4.0 * k / 1024 for k in (1024, -1024, 1, -3, 511, 777, 0, -1000)]
    assert np.array_equal(_reals(oracle.fp16_storage(_site(vals)))[:8], vals)
    # a site of zeros stays zero (scale 0); the other 15 sites are zero sites
    out = oracle.fp16_storage(_site(vals))
    assert np.count_nonzero(out.reshape(16, 12)[1:]) == 0


def test_fp16_storage_ties_to_even_and_subnormals():
    # scale 1: the FP16 spacing in [0.5, 1) is 2^-11
    vals = [1.0,
            0.5 + 2 ** -12,          # tie between 0.5 (even) and 0.5 + 2^-11: 0.5
            0.5 + 3 * 2 ** -12,      # tie between 0.5 + 2^-11 and 0.5 + 2^-10 (even)
            0.5 + 2 ** -12 + 2 ** -20,   # just above the tie: rounds up
            2 ** -20,                # FP16 subnormal (spacing 2^-24), exact
            0.75 * 2 ** -24,         # rounds to the smallest subnormal 2^-24
            0.25 * 2 ** -24]         # rounds to zero
    got = _reals(oracle.fp16_storage(_site(vals)))[:7]
    assert list(got) == [1.0, 0.5, 0.5 + 2 ** -10, 0.5 + 2 ** -11, 2 ** -20, 2 ** -24, 0.0]


def test_fp16_storage_error_bound_and_scale_component():
    # per site: |decoded - v| <= s (2^-12 + 2^-22), half the FP16 spacing in
    # [0.5, 1) plus the FP32 roundings; and the largest component
    # decodes to itself exactly (v r rounds to +-1 in FP16, then 1 * s = s)
    psi = synth.gaussian_source((4, 4, 4, 4), 31) * 1e3
    v32 = oracle.fp32_storage(psi).reshape(-1, 12)
    dec = oracle.fp16_storage(psi).reshape(-1, 12)
    r = lambda a: np.stack([a.real, a.imag], axis=-1).reshape(-1, 24)
    v, d = r(v32), r(dec)
    s = np.abs(v).max(axis=1)
    err = np.abs(d - v).max(axis=1)
    assert np.all(err <= s * (2 ** -12 + 2 ** -22))
    k = np.abs(v).argmax(axis=1)
    rows = np.arange(len(k))
    assert np.array_equal(d[rows, k], v[rows, k])
    # the bound is nearly attained somewhere: the format is not a finer one
    assert (err / s).max() > 0.9 * 2 ** -12
