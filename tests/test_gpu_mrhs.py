"""The multi-system stencil (several sources on one gauge field, Sec. II-A):
MULT (eq. 9) and D-hat_ee (eq. 8) applied to up to 16 fields in one launch,
each thread taking one site for 2 or 4 fields, against the oracle field by
field, against the one-field kernel, and inside batched solves.

Lattices: a ragged one whose parity does not fill its last 64-site tile
(6x6x6x10: 1080 sites per parity), the non-cubic 4x6x8x10, and sampled sites
of the 32^3x64 benchmark lattice with the 12 fields of the point-source batch.
Field counts 2, 5, 12 and 16 leave the last group of 4 (or 2) partly empty.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_checks import check_true_residual, rel, say, site_errors  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402

TOL = {wc.FP64: 1e-13, wc.FP32: 1e-5, wc.FP16: 2e-3}
# batched against one-field results: equal up to the rounding of the stored output
SAME = {wc.FP64: 1e-14, wc.FP32: 1e-6, wc.FP16: 2e-3}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


_cache = {}


def setup(dims, kappa=0.13, csw=1.0, seed=1300):
    key = (dims, kappa, csw, seed)
    if key not in _cache:
        U = synth.random_links(dims, 0.3, seed)
        lat = wc.Lattice(dims)
        lat.load_links(dev(U))
        lat.build_clover(kappa, csw)
        F = oracle.clover_field(U, dims, kappa, csw)
        _cache[key] = (lat, U, oracle.site_invert(F))
    return _cache[key]


# FP64 batches take the one-system-per-thread path (fields' workgroups interleaved)
@pytest.mark.parametrize("prec,recon", [(wc.FP32, 12), (wc.FP32, 8), (wc.FP32, 18), (wc.FP16, 12), (wc.FP64, 12)])
@pytest.mark.parametrize("g", [2, 4, 0])
@pytest.mark.parametrize("dims", [(6, 6, 6, 10), (4, 6, 8, 10)])
def test_mult_batch_against_oracle_and_single(dims, g, prec, recon):
    lat, U, Finv = setup(dims)
    lat.set_link_recon(recon)
    lat.set_multi_rhs(g)
    try:
        for n in (2, 5, 12, 16):
            say("MULT batch", dims, "G", g, "prec", prec, "recon", recon, "fields", n)
            psis = [synth.gaussian_source(dims, 1400 + k) for k in range(n)]
            for out_par in (0, 1):
                eo_in = [lat.pack(dev(p), prec) for p in psis]
                eo_out = [lat.new_eo(prec, 2) for _ in range(n)]
                lat.apply_mult_batch([lat.parity_view(o, out_par, prec) for o in eo_out],
                                     [lat.parity_view(e, 1 - out_par, prec) for e in eo_in], out_par, prec)
                one = lat.new_eo(prec, 2)
                for k in range(n):
                    out = host(lat.unpack(eo_out[k], prec))
                    ref = oracle.htilde(U, Finv, psis[k], out_par)
                    assert rel(out, ref) < TOL[prec], (k, out_par)
                    # the same field through the one-field kernel: equal up to
                    # the rounding of the stored output
                    lat.apply_mult(lat.parity_view(one, out_par, prec), lat.parity_view(eo_in[k], 1 - out_par, prec),
                                   out_par, prec)
                    assert rel(out, host(lat.unpack(one, prec))) < SAME[prec], (k, out_par)
    finally:
        lat.set_link_recon(12)
        lat.set_multi_rhs(-1)


@pytest.mark.parametrize("prec", [wc.FP32, wc.FP16, wc.FP64])
@pytest.mark.parametrize("g", [2, 4])
def test_dhat_batch_against_oracle(g, prec):
    dims = (6, 6, 6, 10)
    kappa = 0.13
    lat, U, Finv = setup(dims, kappa=kappa)
    lat.set_multi_rhs(g)
    try:
        n = 7
        psis = [oracle.restrict(synth.gaussian_source(dims, 1500 + k), 0) for k in range(n)]
        eo_in = [lat.pack(dev(p), prec) for p in psis]
        eo_out = [lat.new_eo(prec, 2) for _ in range(n)]
        lat.apply_Dee_oo_batch([lat.parity_view(o, 0, prec) for o in eo_out],
                               [lat.parity_view(e, 0, prec) for e in eo_in], prec)
        for k in range(n):
            out = host(lat.unpack(eo_out[k], prec))
            ref = oracle.dhat_ee(U, Finv, kappa, psis[k])
            assert rel(out, ref) < TOL[prec], k
    finally:
        lat.set_multi_rhs(-1)


@pytest.mark.parametrize("g", [2, 4, 0])
def test_batched_solves_against_oracle(g):
    # the systems of a batch stop at different iterations (sources of different
    # size and shape), so the groups of the multi-system stencil lose members
    # mid-chunk and are regrouped between chunks
    dims = (6, 6, 6, 10)
    kappa, csw = 0.13, 1.0
    lat, U, Finv = setup(dims, kappa=kappa, csw=csw)
    lat.set_multi_rhs(g)
    try:
        bs = [synth.gaussian_source(dims, 1600 + k) * (10.0 ** (k % 3 - 1)) for k in range(9)]
        bs[4] = synth.point_source(dims, 2, 1)
        F = oracle.clover_field(U, dims, kappa, csw)
        for inner in (wc.FP32, wc.FP16):
            xs, infos = lat.solve_batch([dev(b) for b in bs], kappa, csw, 1e-11, inner_prec=inner)
            say("G", g, "inner", inner, [i["inner_iters_total"] for i in infos])
            for k in range(len(bs)):
                check_true_residual(U, kappa, csw, bs[k], host(xs[k]), infos[k], 1e-11)
            x_ref, _, _ = oracle.solve(U, F, kappa, bs[0], tol=1e-13)
            assert rel(host(xs[0]), x_ref) < 1e-9
    finally:
        lat.set_multi_rhs(-1)


def test_settings_are_checked():
    lat, _, _ = setup((6, 6, 6, 10))
    for bad in (1, 3, 8, -2):
        with pytest.raises(wc.WCError):
            lat.set_multi_rhs(bad)
    assert lat.multi_rhs(wc.FP32) == 2 and lat.multi_rhs(wc.FP16) == 4 and lat.multi_rhs(wc.FP64) == 0
    lat.set_multi_rhs(4)
    assert lat.multi_rhs(wc.FP32) == 4
    lat.set_multi_rhs(-1)
    for bad in (-2, 1 << 21):
        with pytest.raises(wc.WCError):
            lat.set_xcd_chunk(bad)
    lat.set_xcd_chunk(0)
    assert lat.xcd_chunk(wc.FP32) == 0 and lat.xcd_chunk(wc.FP16) == 0
    lat.set_xcd_chunk(-1)


@pytest.mark.timeout(600)
def test_mult_batch_sampled_sites_32x32x32x64():
    # the 12 fields of the point-source batch's size at the benchmark's lattice
    dims = (32, 32, 32, 64)
    kappa, csw = 0.135, 1.0
    Ud = synth.random_links_torch(dims, 0.3, 1004, device="cuda")
    lat = wc.Lattice(dims)
    lat.load_links(Ud)
    lat.build_clover(kappa, csw)
    U = Ud.cpu().numpy()
    del Ud
    n = 12
    prec = wc.FP32
    V = int(np.prod(dims))
    par = oracle.parity(dims).reshape(-1)
    g = synth.rng(17)
    cand = np.concatenate([g.integers(0, V, 2000), [0, 1, V - 2, V - 1, dims[0] - 1]])
    sites = np.unique(cand[par[cand] == 0])
    eo_in, eo_out, psis = [], [], []
    for k in (0, 5, 11):
        psis.append(synth.gaussian_source(dims, 1700 + k))
    for k in range(n):
        eo_in.append(lat.pack(dev(psis[[0, 5, 11].index(k)] if k in (0, 5, 11) else psis[0] * (k + 1)), prec))
        eo_out.append(lat.new_eo(prec, 2))
    lat.apply_mult_batch([lat.parity_view(o, 0, prec) for o in eo_out], [lat.parity_view(e, 1, prec) for e in eo_in],
                         0, prec)
    for j, k in enumerate((0, 5, 11)):
        out = host(lat.unpack(eo_out[k], prec)).reshape(-1, 4, 3)
        ref = oracle.htilde_sites(U, kappa, csw, psis[j], sites)
        err, _ = site_errors(out[sites], ref, "12-field MULT, field %d" % k)
        assert err < 1e-5, k
    lat.close()
    torch.cuda.empty_cache()
