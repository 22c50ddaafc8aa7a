"""The waves-per-CU cap of the one-system stencils: MULT (Sec. II-B eq. 9),
D-hat_ee (eq. 8) and D (eqs. 3-4) give bit-identical results under every cap
and block size, and the cap's settings are checked.

The cap only reserves LDS that the kernels do not touch, so the arithmetic and
its order are the same; the results are compared byte for byte with the
uncapped launch, and once against the oracle.  Lattice 6x6x6x10 leaves the
last 64-site tile of each parity partly empty (1080 sites per parity).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_checks import rel, say  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402

TOL = {wc.FP64: 1e-13, wc.FP32: 1e-5, wc.FP16: 2e-3}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


_cache = {}


def setup(dims=(6, 6, 6, 10), kappa=0.13, csw=1.0, seed=1800):
    key = (dims, kappa, csw, seed)
    if key not in _cache:
        U = synth.random_links(dims, 0.3, seed)
        lat = wc.Lattice(dims)
        lat.load_links(dev(U))
        lat.build_clover(kappa, csw)
        F = oracle.clover_field(U, dims, kappa, csw)
        _cache[key] = (lat, U, oracle.site_invert(F))
    return _cache[key]


def test_defaults_and_settings():
    lat, _, _ = setup()
    caps = (lat.wave_cap(wc.FP64), lat.wave_cap(wc.FP32), lat.wave_cap(wc.FP16))
    say("default caps", caps)
    assert caps == (8, 0, 0)
    assert lat.wave_cap(wc.FP64, dhat=True) == 8 and lat.wave_cap(wc.FP32, dhat=True) == 0
    for bad in (-2, 1, 2, 3, 5, 20, 32, 64):
        with pytest.raises(wc.WCError):
            lat.set_wave_cap(wc.FP64, bad)
    with pytest.raises(wc.WCError):
        lat.set_wave_cap(3, 8)
    lat.set_wave_cap(wc.FP32, 12)
    assert lat.wave_cap(wc.FP32) == 12 and lat.wave_cap(wc.FP32, dhat=True) == 12 and lat.wave_cap(wc.FP64) == 8
    lat.set_wave_cap(wc.FP64, 0)
    assert lat.wave_cap(wc.FP64) == 0
    lat.set_wave_cap(wc.FP32, -1)
    lat.set_wave_cap(wc.FP64, -1)
    assert lat.wave_cap(wc.FP64) == 8 and lat.wave_cap(wc.FP32) == 0


@pytest.mark.parametrize("prec,recon", [(wc.FP64, 12), (wc.FP32, 12), (wc.FP32, 8), (wc.FP32, 18),
                                        (wc.FP16, 12)])
def test_results_identical_under_every_cap_and_block_size(prec, recon):
    # FP32 in each link form: the reconstruct-8 stencil loads both hops of a
    # direction before rebuilding either link, at four waves per SIMD
    dims, kappa = (6, 6, 6, 10), 0.13
    lat, U, Finv = setup(dims, kappa)
    psi = synth.gaussian_source(dims, 1810)
    try:
        lat.set_link_recon(recon)
        eo = lat.pack(dev(psi), prec)
        for bs in (64, 128, 256):
            lat.set_block_size(bs)
            ref = None
            for cap in (0, 4, 8, 12, 16, -1):
                lat.set_wave_cap(prec, cap)
                say("prec", prec, "links", recon, "threads", bs, "cap", cap, "->", lat.wave_cap(prec))
                m = lat.new_eo(prec, 2)
                lat.apply_mult(lat.parity_view(m, 0, prec), lat.parity_view(eo, 1, prec), 0, prec)
                lat.apply_mult(lat.parity_view(m, 1, prec), lat.parity_view(eo, 0, prec), 1, prec)
                d = lat.new_eo(prec, 2)
                lat.apply_Dee_oo(lat.parity_view(d, 0, prec), lat.parity_view(eo, 0, prec), prec)
                full = host(lat.apply_D(dev(psi), prec)) if prec != wc.FP16 else None
                got = (host(m).tobytes(), host(d)[:lat.spinor_bytes(prec)].tobytes(),
                       None if full is None else full.tobytes())
                if ref is None:
                    ref = got
                    # the uncapped launch against the oracle
                    out = host(lat.unpack(m, prec))
                    for par in (0, 1):
                        want = oracle.htilde(U, Finv, oracle.restrict(psi, 1 - par), par)
                        assert rel(oracle.restrict(out, par), want) < TOL[prec], par
                else:
                    assert got == ref, (bs, cap)
    finally:
        lat.set_block_size(0)
        lat.set_wave_cap(prec, -1)
        lat.set_link_recon(12)


def test_fp64_solve_under_no_cap_and_tuned_cap_agree():
    # the launch shape pinned, so that only the cap differs between the solves
    dims, kappa, csw = (6, 6, 6, 10), 0.13, 1.0
    lat, U, _ = setup(dims, kappa, csw)
    b = synth.gaussian_source(dims, 1820)
    xs = []
    try:
        lat.set_block_size(128)
        lat.set_xcd_chunk(16)
        for cap in (0, 12, -1):
            lat.set_wave_cap(wc.FP64, cap)
            x, info = lat.solve(dev(b), kappa, csw, 1e-12, inner_prec=wc.FP64)
            say("cap", cap, "->", lat.wave_cap(wc.FP64), lat.wave_cap(wc.FP64, dhat=True),
                "iterations", info["inner_iters_total"])
            r, bn = oracle.residual(U, kappa, csw, b, host(x))
            assert r / bn < 1e-12
            xs.append(host(x))
        assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    finally:
        lat.set_wave_cap(wc.FP64, -1)
        lat.set_block_size(0)
        lat.set_xcd_chunk(-1)


@pytest.mark.parametrize("prec", [wc.FP64, wc.FP32, wc.FP16])
def test_tuner_picks_valid_caps_per_kernel_class(prec):
    dims = (8, 8, 8, 16)
    U = synth.random_links(dims, 0.3, 1830)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    lat.build_clover(0.13, 1.0)
    r = lat.tune_block_size(prec)
    say("prec", prec, r)
    for v in r["wave_cap"].values():
        assert v in (0, 8, 12)
    assert r["wave_cap"]["mult"] == lat.wave_cap(prec) and r["wave_cap"]["dhat"] == lat.wave_cap(prec, dhat=True)
    # a pinned cap is not tuned
    lat.set_wave_cap(prec, 16)
    r = lat.tune_block_size(prec)
    assert r["wave_cap"] == {"mult": 16, "dhat": 16}
    lat.close()
