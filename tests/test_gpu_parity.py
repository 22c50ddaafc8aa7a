"""GPU parity: every kernel of the HIP path against the FP64 oracle, element by
element, on seeded inputs (non-cubic extents to catch axis swaps, 2^4 for the
degenerate wrap where n + mu = n - mu, ragged volumes that do not fill the
last 256-thread block).

Tolerances: FP64 paths agree to rounding (1e-13 relative); single FP32
operator applications to 1e-5 relative (the FP32 bound; FP32 rounding over
the ~100 terms of one output is ~1e-6); FP16 storage to 2e-3 relative (half
precision keeps 11 significant bits, ~5e-4 per stored value).  Solutions of
the FP64-refined solves agree with the oracle's to 1e-10.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_checks import check_true_residual, rel  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU but never run there
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402

TOL = {wc.FP64: 1e-13, wc.FP32: 1e-5, wc.FP16: 2e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


_cache = {}


def setup_case(dims, seed=1000, kappa=0.13, csw=1.0, kind="random"):
    key = (dims, seed, kappa, csw, kind)
    if key in _cache:
        return _cache[key]
    if kind == "random":
        U = synth.random_links(dims, 0.3, seed)
    elif kind == "unit":
        U = synth.unit_links(dims)
    else:
        lx, ly, lz, lt = dims
        om = synth.haar_su3((lt, lz, ly, lx), synth.rng(seed))
        U = synth.pure_gauge_links(om, dims)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    lat.build_clover(kappa, csw)
    F = oracle.clover_field(U, dims, kappa, csw)
    Finv = oracle.site_invert(F)
    out = (lat, U, F, Finv)
    _cache[key] = out
    return out


DIMS = [(4, 6, 8, 10), (2, 2, 2, 2), (6, 4, 2, 8), (8, 8, 8, 8)]
PRECS = [wc.FP64, wc.FP32, wc.FP16]


def storage_cases(dims, seed):
    """A Gaussian field whose first sites hold the storage formats' special
    cases: a zero site; FP16 ties, a value just above a tie and FP16
    subnormals (scale 8); and sites scaled by 1e-30 and 1e30."""
    psi = synth.gaussian_source(dims, seed)
    f = psi.reshape(-1, 12)
    f[0] = 0
    vals = 8.0 * np.array([1.0, 0.5 + 2 ** -12, 0.5 + 3 * 2 ** -12, 0.5 + 2 ** -12 + 2 ** -20,
                           2 ** -20, 0.75 * 2 ** -24, 0.25 * 2 ** -24, -1.0] + [0.0] * 16)
    f[1] = vals[0::2] + 1j * vals[1::2]
    f[2] *= 1e-30
    f[3] *= 1e30
    return psi


STORED = {wc.FP64: lambda a: a, wc.FP32: oracle.fp32_storage, wc.FP16: oracle.fp16_storage}


def assert_bits_equal(got, want):
    bad = np.argwhere(got != want)
    assert bad.size == 0, (len(bad), [(tuple(i), got[tuple(i)], want[tuple(i)]) for i in bad[:4]])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", DIMS[:3])
def test_pack_unpack_roundtrip(dims, prec):
    # the stored copy reads back bit for bit as the oracle's storage model:
    # FP64 unchanged, FP32 rounded to nearest even, FP16 with the per-site scale
    say("pack", dims, prec)
    lat, U, F, Finv = setup_case(dims)
    psi = storage_cases(dims, 5)
    back = host(lat.unpack(lat.pack(dev(psi), prec), prec))
    assert_bits_equal(back, STORED[prec](psi))


@pytest.mark.parametrize("prec", [wc.FP64, wc.FP32])
@pytest.mark.parametrize("dims", DIMS)
def test_apply_D(dims, prec):
    say("apply_D", dims, prec)
    kappa = 0.13
    lat, U, F, Finv = setup_case(dims, kappa=kappa)
    psi = synth.gaussian_source(dims, 7)
    ref = oracle.apply_D(U, F, kappa, psi)
    out = host(lat.apply_D(dev(psi), prec))
    assert rel(out, ref) < TOL[prec]


@pytest.mark.parametrize("kind", ["unit", "pure"])
def test_apply_D_trivial_gauge(kind):
    dims = (4, 6, 8, 10)
    say("apply_D", kind)
    lat, U, F, Finv = setup_case(dims, seed=3, kind=kind)
    psi = synth.gaussian_source(dims, 8)
    ref = oracle.apply_D(U, F, 0.13, psi)
    assert rel(host(lat.apply_D(dev(psi), wc.FP64)), ref) < 1e-13


def _eo_single(lat, prec, psi, parity):
    """Pack psi and return (two-parity buffer, view of the requested parity)."""
    eo = lat.pack(dev(psi), prec)
    return eo, lat.parity_view(eo, parity, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", DIMS[:3])
def test_clover_and_inverse(dims, prec):
    say("clover", dims, prec)
    lat, U, F, Finv = setup_case(dims, kappa=0.1355)
    psi = synth.gaussian_source(dims, 9)
    eo_in = lat.pack(dev(psi), prec)
    for inverse, M in [(0, F), (1, Finv)]:
        for parity in (0, 1):
            eo_out = lat.new_eo(prec, 2)
            lat.apply_clover(lat.parity_view(eo_out, parity, prec), lat.parity_view(eo_in, parity, prec), parity,
                             inverse, prec)
            out = host(lat.unpack(eo_out, prec))
            ref = oracle.restrict(oracle.site_apply(M, psi), parity)
            tol = TOL[prec] if prec != wc.FP16 else 3e-3
            assert rel(out, ref) < tol, (inverse, parity)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", DIMS)
def test_mult_both_parities(dims, prec):
    say("mult", dims, prec)
    lat, U, F, Finv = setup_case(dims)
    psi = synth.gaussian_source(dims, 10)
    eo_in = lat.pack(dev(psi), prec)
    for out_par in (0, 1):
        eo_out = lat.new_eo(prec, 2)
        lat.apply_mult(lat.parity_view(eo_out, out_par, prec), lat.parity_view(eo_in, 1 - out_par, prec), out_par,
                       prec)
        out = host(lat.unpack(eo_out, prec))
        ref = oracle.htilde(U, Finv, psi, out_par)
        assert rel(out, ref) < TOL[prec], out_par


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", DIMS)
def test_dhat_ee(dims, prec):
    say("dhat", dims, prec)
    kappa = 0.13
    lat, U, F, Finv = setup_case(dims, kappa=kappa)
    psi = oracle.restrict(synth.gaussian_source(dims, 11), 0)
    eo_in = lat.pack(dev(psi), prec)
    eo_out = lat.new_eo(prec, 2)
    lat.apply_Dee_oo(lat.parity_view(eo_out, 0, prec), lat.parity_view(eo_in, 0, prec), prec)
    out = host(lat.unpack(eo_out, prec))
    ref = oracle.dhat_ee(U, Finv, kappa, psi)
    assert rel(out, ref) < TOL[prec]


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP64, wc.FP16])
def test_solve_8x4_matches_oracle(inner):
    # the 8^4, kappa = 0.12 case: oracle solution to 1e-13, GPU to 1e-12
    dims = (8, 8, 8, 8)
    kappa, csw = 0.12, 1.0
    say("solve 8^4", inner)
    lat, U, F, Finv = setup_case(dims, seed=1001, kappa=kappa, csw=csw)
    b = synth.gaussian_source(dims, 2001)
    x_ref, it, rr = oracle.solve(U, F, kappa, b, tol=1e-13)
    x, info = lat.solve(dev(b), kappa, csw, 1e-12, inner_prec=inner)
    x = host(x)
    say(info)
    r, bn = oracle.residual(U, kappa, csw, b, x)
    assert r / bn < 1e-12
    assert info["true_rel_residual"] < 1e-12
    assert abs(info["true_rel_residual"] - r / bn) < 1e-13
    assert rel(x, x_ref) < 1e-10


@pytest.mark.parametrize("kappa", [0.135, 0.1355])
def test_solve_near_critical_kappas(kappa):
    dims = (8, 8, 8, 16)
    say("solve", dims, kappa)
    lat, U, F, Finv = setup_case(dims, seed=1002, kappa=kappa)
    b = synth.gaussian_source(dims, 2002)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-10)
    say(info)
    check_true_residual(U, kappa, 1.0, b, host(x), info, 1e-10)


def test_solve_pure_gauge_fft_closed_form():
    # D[U] = Om D_free Om^dagger: x = Om FFT-solve(Om^dagger b), no oracle solver needed
    dims = (8, 8, 8, 16)
    kappa = 0.12
    lx, ly, lz, lt = dims
    om = synth.haar_su3((lt, lz, ly, lx), synth.rng(77))
    U = synth.pure_gauge_links(om, dims)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    b = synth.gaussian_source(dims, 78)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12)
    omd_b = np.einsum("...ji,...aj->...ai", np.conj(om), b)
    x_ref = np.einsum("...ij,...aj->...ai", om, oracle.free_solve_fft(omd_b, kappa))
    assert rel(host(x), x_ref) < 1e-10


def test_solve_gauge_covariance():
    # x[U^Om, Om b] = Om x[U, b] for U^Om_mu(n) = Om(n) U_mu(n) Om(n+mu)^dagger
    dims = (8, 8, 8, 16)
    kappa = 0.13
    lx, ly, lz, lt = dims
    U = synth.random_links(dims, 0.3, 1020)
    om = synth.haar_su3((lt, lz, ly, lx), synth.rng(1021))
    Uo = synth.gauge_transform_links(U, om, dims)
    b = synth.gaussian_source(dims, 1022)
    bo = np.einsum("...ij,...aj->...ai", om, b)
    xs = []
    for links, src in ((U, b), (Uo, bo)):
        lat = wc.Lattice(dims)
        lat.load_links(dev(links))
        x, info = lat.solve(dev(src), kappa, 1.0, 1e-12)
        assert info["true_rel_residual"] < 1e-12
        xs.append(host(x))
        lat.close()
    assert rel(xs[1], np.einsum("...ij,...aj->...ai", om, xs[0])) < 1e-10


def test_solve_zero_source_and_guess():
    dims = (4, 4, 4, 4)
    lat, U, F, Finv = setup_case(dims, seed=5)
    z = np.zeros(synth.shape_spinor(dims), dtype=np.complex128)
    x, info = lat.solve(dev(z), 0.13, 1.0, 1e-10)
    assert np.all(host(x) == 0)
    b = synth.gaussian_source(dims, 6)
    x_ref, _, _ = oracle.solve(U, F, 0.13, b, tol=1e-13)
    x, info = lat.solve(dev(b), 0.13, 1.0, 1e-11, x0=dev(x_ref))
    assert info["true_rel_residual"] < 1e-11
    assert info["inner_calls"] <= 2


def test_solve_fixed_work_mode():
    dims = (4, 4, 4, 8)
    lat, U, F, Finv = setup_case(dims, seed=9)
    b = synth.gaussian_source(dims, 10)
    x, info = lat.solve(dev(b), 0.13, 1.0, 1e-10, fixed_work=20, raise_on_error=False)
    assert info["inner_iters_total"] == 20 * info["inner_calls"]
