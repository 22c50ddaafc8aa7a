"""Parity at the full benchmark sizes: the operator on sampled output sites
against the oracle's site-by-site D, MULT, D-hat_ee and clover blocks (relative
L2 error and the largest per-site error printed), and complete solves checked
through the oracle's FP64 true residual on the whole lattice, which must also
agree with the residual the library reports.  One 32^3x64 solution is compared
with the oracle's own solve of the same system, and pure-gauge systems with
the momentum-space closed form."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_checks import check_true_residual, say, site_errors  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


@pytest.fixture(scope="module")
def c2():
    dims = (32, 32, 32, 64)
    Ud = synth.random_links_torch(dims, 0.3, 1002, device="cuda")
    lat = wc.Lattice(dims)
    lat.load_links(Ud)
    lat.build_clover(0.135, 1.0)
    U = Ud.cpu().numpy()
    return dims, lat, U, Ud


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5)])
def test_apply_D_sampled_sites_32x32x32x64(c2, prec, tol):
    dims, lat, U, Ud = c2
    say("apply_D sampled", prec)
    psi = synth.gaussian_source(dims, 2002)
    out = lat.apply_D(torch.from_numpy(psi).cuda(), prec).cpu().numpy().reshape(-1, 4, 3)
    g = synth.rng(9)
    V = int(np.prod(dims))
    sites = np.concatenate([g.integers(0, V, 4000), [0, 1, V - 1, V - 2, dims[0] - 1]])
    ref = oracle.apply_D_sites(U, 0.135, 1.0, psi, sites)
    err, _ = site_errors(out[sites], ref, "apply_D")
    assert err < tol


@pytest.mark.parametrize("prec", [wc.FP32, wc.FP16])
def test_pack_unpack_bit_exact_32x32x32x64(c2, prec):
    # every site of the full lattice reads back as the oracle's storage model
    dims, lat, U, Ud = c2
    say("pack/unpack 32^3x64", prec)
    psi = synth.gaussian_source(dims, 2003)
    back = lat.unpack(lat.pack(torch.from_numpy(psi).cuda(), prec), prec).cpu().numpy()
    want = (oracle.fp32_storage if prec == wc.FP32 else oracle.fp16_storage)(psi)
    bad = int(np.count_nonzero(back != want))
    say("mismatched reals", bad)
    assert bad == 0


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5), (wc.FP16, 2e-3)])
def test_dhat_ee_sampled_even_sites_32x32x32x64(c2, prec, tol):
    # D-hat_ee, the inner loop's operator, at the benchmark's lattice and
    # launch shape against the oracle's site-by-site D-hat_ee (eq. 8)
    dims, lat, U, Ud = c2
    kappa, csw = 0.135, 1.0
    say("D-hat_ee sampled", prec)
    psi = oracle.restrict(synth.gaussian_source(dims, 2004), 0)
    eo_in = lat.pack(torch.from_numpy(psi).cuda(), prec)
    eo_out = lat.new_eo(prec, 2)
    lat.apply_Dee_oo(lat.parity_view(eo_out, 0, prec), lat.parity_view(eo_in, 0, prec), prec)
    out = lat.unpack(eo_out, prec).cpu().numpy().reshape(-1, 4, 3)
    even = oracle.parity(dims).reshape(-1) == 0
    V = int(np.prod(dims))
    g = synth.rng(10)
    cand = np.concatenate([g.integers(0, V, 6000), [0, 1, 2, V // 2, V - 2, V - 1, dims[0] - 2, dims[0] - 1]])
    sites = np.unique(cand[even[cand]])
    ref = oracle.dhat_ee_sites(U, kappa, csw, psi, sites)
    err, _ = site_errors(out[sites], ref, "D-hat_ee even")
    assert err < tol


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5), (wc.FP16, 3e-3)])
def test_clover_and_inverse_sampled_sites_32x32x32x64(c2, prec, tol):
    # the stored clover blocks F and F^-1 of each parity against the oracle's F
    # built site by site from the links
    dims, lat, U, Ud = c2
    kappa, csw = 0.135, 1.0
    psi = synth.gaussian_source(dims, 2006)
    eo_in = lat.pack(torch.from_numpy(psi).cuda(), prec)
    par = oracle.parity(dims).reshape(-1)
    V = int(np.prod(dims))
    g = synth.rng(14)
    cand = np.concatenate([g.integers(0, V, 4000), [0, 1, V - 2, V - 1]])
    for inverse in (0, 1):
        for p in (0, 1):
            eo_out = lat.new_eo(prec, 2)
            lat.apply_clover(lat.parity_view(eo_out, p, prec), lat.parity_view(eo_in, p, prec), p, inverse, prec)
            out = lat.unpack(eo_out, prec).cpu().numpy().reshape(-1, 4, 3)
            sites = np.unique(cand[par[cand] == p])
            ref = oracle.clover_sites(U, kappa, csw, psi, sites, bool(inverse))
            err, _ = site_errors(out[sites], ref, "clover prec %d inverse %d parity %d" % (prec, inverse, p))
            assert err < tol, (inverse, p)


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5), (wc.FP16, 2e-3)])
def test_mult_sampled_sites_both_parities_32x32x32x64(c2, prec, tol):
    # MULT = F^-1 H into each parity, against the oracle's site-by-site MULT
    dims, lat, U, Ud = c2
    kappa, csw = 0.135, 1.0
    psi = synth.gaussian_source(dims, 2005)
    eo_in = lat.pack(torch.from_numpy(psi).cuda(), prec)
    par = oracle.parity(dims).reshape(-1)
    V = int(np.prod(dims))
    g = synth.rng(12)
    cand = np.concatenate([g.integers(0, V, 6000), [0, 1, 2, V // 2, V - 2, V - 1, dims[0] - 2, dims[0] - 1]])
    for p in (0, 1):
        say("MULT sampled", prec, "into parity", p)
        eo_out = lat.new_eo(prec, 2)
        lat.apply_mult(lat.parity_view(eo_out, p, prec), lat.parity_view(eo_in, 1 - p, prec), p, prec)
        out = lat.unpack(eo_out, prec).cpu().numpy().reshape(-1, 4, 3)
        sites = np.unique(cand[par[cand] == p])
        ref = oracle.htilde_sites(U, kappa, csw, psi, sites)
        err, _ = site_errors(out[sites], ref, "MULT")
        assert err < tol, p


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP16])
def test_solve_32x32x32x64_oracle_residual(c2, inner):
    dims, lat, U, Ud = c2
    say("solve 32^3x64", inner)
    b = synth.gaussian_source(dims, 2002)
    x, info = lat.solve(torch.from_numpy(b).cuda(), 0.135, 1.0, 1e-10, inner_prec=inner)
    say(info)
    check_true_residual(U, 0.135, 1.0, b, x.cpu().numpy(), info, 1e-10)


@pytest.mark.parametrize("recon", [8, 18])
def test_apply_D_other_link_forms_sampled_sites_32x32x32x64(c2, recon):
    dims, lat, U, Ud = c2
    say("apply_D sampled, link form", recon)
    psi = synth.gaussian_source(dims, 2002)
    lat.set_link_recon(recon)
    try:
        out = lat.apply_D(torch.from_numpy(psi).cuda(), wc.FP32).cpu().numpy().reshape(-1, 4, 3)
    finally:
        lat.set_link_recon(12)
    g = synth.rng(10)
    V = int(np.prod(dims))
    sites = np.concatenate([g.integers(0, V, 4000), [0, 1, V - 1, V - 2, dims[0] - 1]])
    ref = oracle.apply_D_sites(U, 0.135, 1.0, psi, sites)
    err, _ = site_errors(out[sites], ref, "apply_D recon %d" % recon)
    assert err < 1e-5


@pytest.mark.parametrize("inner,recon,outer", [(wc.FP32, 8, "bicgstab"), (wc.FP16, 12, "dc")])
def test_solve_32x32x32x64_variants_oracle_residual(c2, inner, recon, outer):
    dims, lat, U, Ud = c2
    say("solve 32^3x64", inner, recon, outer)
    b = synth.gaussian_source(dims, 2002)
    lat.set_link_recon(recon)
    try:
        x, info = lat.solve(torch.from_numpy(b).cuda(), 0.135, 1.0, 1e-10, inner_prec=inner, outer=outer)
    finally:
        lat.set_link_recon(12)
    say(info)
    check_true_residual(U, 0.135, 1.0, b, x.cpu().numpy(), info, 1e-10)


@pytest.mark.timeout(900)
def test_solve_32x32x32x64_solution_matches_oracle_solve(c2):
    # the headline system itself: the GPU's nested solve (to 1e-12) against the
    # oracle's plain FP64 BiCGStab on the full D (to 1e-13), solution to 1e-10
    dims, lat, U, Ud = c2
    kappa, csw = 0.135, 1.0
    say("solve 32^3x64 against the oracle's solve (%d host threads)" % oracle.num_threads())
    b = synth.gaussian_source(dims, 2002)
    x, info = lat.solve(torch.from_numpy(b).cuda(), kappa, csw, 1e-12)
    say(info)
    xh = x.cpu().numpy()
    del x
    check_true_residual(U, kappa, csw, b, xh, info, 1e-12)
    F = oracle.clover_field(U, dims, kappa, csw)
    x_ref, its, rr = oracle.solve(U, F, kappa, b, tol=1e-13)
    del F
    err = float(np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref))
    say("oracle: %d iterations, true rel residual %.3e; solution rel err %.3e" % (its, rr, err))
    site_errors(xh.reshape(-1, 4, 3), x_ref.reshape(-1, 4, 3), "solution")
    assert err < 1e-10


@pytest.fixture(scope="module")
def c3():
    dims = (48, 48, 48, 96)
    Ud = synth.random_links_torch(dims, 0.3, 1003, device="cuda")
    lat = wc.Lattice(dims)
    lat.load_links(Ud)
    U = Ud.cpu().numpy()
    del Ud
    b = synth.z2_source(dims, 2003)
    yield dims, lat, U, b
    lat.close()


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5)])
def test_apply_D_sampled_sites_48x48x48x96(c3, prec, tol):
    # the precision-comparison lattice: random sites, both ends of the site
    # order and of each parity slab, and the last x and t slices
    dims, lat, U, b = c3
    kappa, csw = 0.1355, 1.0
    lat.build_clover(kappa, csw)
    say("apply_D sampled 48^3x96", prec)
    psi = synth.gaussian_source(dims, 2013)
    out = lat.apply_D(torch.from_numpy(psi).cuda(), prec).cpu().numpy().reshape(-1, 4, 3)
    V = int(np.prod(dims))
    g = synth.rng(13)
    sites = np.concatenate([g.integers(0, V, 4000), [0, 1, V // 2 - 1, V // 2, V - 2, V - 1, dims[0] - 1,
                                                     V - dims[0] * dims[1] * dims[2]]])
    ref = oracle.apply_D_sites(U, kappa, csw, psi, sites)
    err, _ = site_errors(out[sites], ref, "apply_D 48^3x96")
    assert err < tol


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5), (wc.FP16, 2e-3)])
def test_dhat_ee_sampled_even_sites_48x48x48x96(c3, prec, tol):
    dims, lat, U, b = c3
    kappa, csw = 0.1355, 1.0
    lat.build_clover(kappa, csw)
    say("D-hat_ee sampled 48^3x96", prec)
    psi = oracle.restrict(synth.gaussian_source(dims, 2014), 0)
    eo_in = lat.pack(torch.from_numpy(psi).cuda(), prec)
    eo_out = lat.new_eo(prec, 2)
    lat.apply_Dee_oo(lat.parity_view(eo_out, 0, prec), lat.parity_view(eo_in, 0, prec), prec)
    out = lat.unpack(eo_out, prec).cpu().numpy().reshape(-1, 4, 3)
    even = oracle.parity(dims).reshape(-1) == 0
    V = int(np.prod(dims))
    g = synth.rng(15)
    cand = np.concatenate([g.integers(0, V, 4000), [0, 2, V // 2, V - 2, V - 1, dims[0] - 2, dims[0] - 1]])
    sites = np.unique(cand[even[cand]])
    ref = oracle.dhat_ee_sites(U, kappa, csw, psi, sites)
    err, _ = site_errors(out[sites], ref, "D-hat_ee even")
    assert err < tol


@pytest.mark.parametrize("prec,tol", [(wc.FP64, 1e-13), (wc.FP32, 1e-5), (wc.FP16, 2e-3)])
def test_mult_sampled_sites_both_parities_48x48x48x96(c3, prec, tol):
    # MULT = F^-1 H into each parity on the precision-comparison lattice
    dims, lat, U, b = c3
    kappa, csw = 0.1355, 1.0
    lat.build_clover(kappa, csw)
    psi = synth.gaussian_source(dims, 2015)
    eo_in = lat.pack(torch.from_numpy(psi).cuda(), prec)
    par = oracle.parity(dims).reshape(-1)
    V = int(np.prod(dims))
    g = synth.rng(16)
    cand = np.concatenate([g.integers(0, V, 4000), [0, 1, 2, V // 2, V - 2, V - 1, dims[0] - 2, dims[0] - 1]])
    for p in (0, 1):
        say("MULT sampled 48^3x96", prec, "into parity", p)
        eo_out = lat.new_eo(prec, 2)
        lat.apply_mult(lat.parity_view(eo_out, p, prec), lat.parity_view(eo_in, 1 - p, prec), p, prec)
        out = lat.unpack(eo_out, prec).cpu().numpy().reshape(-1, 4, 3)
        del eo_out
        sites = np.unique(cand[par[cand] == p])
        ref = oracle.htilde_sites(U, kappa, csw, psi, sites)
        err, _ = site_errors(out[sites], ref, "MULT 48^3x96")
        assert err < tol, p


@pytest.mark.parametrize("inner", [wc.FP16, wc.FP32, wc.FP64])
def test_solve_48x48x48x96_three_forms_oracle_residual(c3, inner):
    # the three precision forms of the 48^3x96 comparison (FP16-storage and FP32
    # inner loops under the FP64 outer, and the all-FP64 BiCGStab), two-column links
    dims, lat, U, b = c3
    kappa, csw = 0.1355, 1.0
    say("solve 48^3x96 inner", inner)
    x, info = lat.solve(torch.from_numpy(b).cuda(), kappa, csw, 1e-10, inner_prec=inner)
    say(info)
    check_true_residual(U, kappa, csw, b, x.cpu().numpy(), info, 1e-10)


def test_solve_48x48x48x96_recon8_converges_like_recon12(c3):
    # 42M links: a link rebuilt from the wrong entries anywhere would slow the
    # FP32 inner solve well beyond the two-column form's 198 iterations
    dims, lat, U, b = c3
    kappa, csw = 0.1355, 1.0
    say("solve 48^3x96 fp32 reconstruct-8")
    lat.set_link_recon(8)
    try:
        x, info = lat.solve(torch.from_numpy(b).cuda(), kappa, csw, 1e-10, inner_prec=wc.FP32)
    finally:
        lat.set_link_recon(12)
    say(info)
    check_true_residual(U, kappa, csw, b, x.cpu().numpy(), info, 1e-10)
    assert info["outer_iters"] == 1 and info["inner_iters_total"] < 230


def test_solve_pure_gauge_fft_32x32x32x64():
    # full-size solve with no oracle solver: for U_mu(n) = Om(n) Om(n+mu)^dagger,
    # D[U] = Om D_free Om^dagger, so x = Om FFT-solve(Om^dagger b) (closed form
    # in momentum space); Haar Om makes every link a generic SU(3) matrix
    dims = (32, 32, 32, 64)
    kappa = 0.12
    lx, ly, lz, lt = dims
    say("pure gauge FFT solve 32^3x64")
    om = synth.haar_su3((lt, lz, ly, lx), synth.rng(78))
    U = synth.pure_gauge_links(om, dims)
    lat = wc.Lattice(dims)
    lat.load_links(torch.from_numpy(U).cuda())
    del U
    b = synth.gaussian_source(dims, 79)
    x, info = lat.solve(torch.from_numpy(b).cuda(), kappa, 1.0, 1e-12)
    say(info)
    omd_b = np.einsum("...ji,...aj->...ai", np.conj(om), b)
    x_ref = np.einsum("...ij,...aj->...ai", om, oracle.free_solve_fft(omd_b, kappa))
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    say("rel err", err)
    assert err < 1e-10
    lat.close()


def test_solve_pure_gauge_fft_48x48x48x96():
    # the closed form at the precision-comparison size (10.6M sites): for
    # U_mu(n) = Om(n) Om(n+mu)^dagger, x = Om FFT-solve(Om^dagger b)
    dims = (48, 48, 48, 96)
    kappa = 0.12
    lx, ly, lz, lt = dims
    say("pure gauge FFT solve 48^3x96")
    om = synth.haar_su3((lt, lz, ly, lx), synth.rng(88))
    U = synth.pure_gauge_links(om, dims)
    lat = wc.Lattice(dims)
    lat.load_links(torch.from_numpy(U).cuda())
    del U
    b = synth.gaussian_source(dims, 89)
    x, info = lat.solve(torch.from_numpy(b).cuda(), kappa, 1.0, 1e-12)
    say(info)
    xh = x.cpu().numpy()
    del x
    lat.close()
    torch.cuda.empty_cache()
    omd_b = np.einsum("...ji,...aj->...ai", np.conj(om), b)
    del b
    x_ref = np.einsum("...ij,...aj->...ai", om, oracle.free_solve_fft(omd_b, kappa))
    del omd_b, om
    err = float(np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref))
    say("rel err", err)
    assert err < 1e-10
