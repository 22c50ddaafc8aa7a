"""The clover blocks' positive-definiteness check (Sec. II-A, F; Sec. II-B, F_ee^-1
and F_oo^-1 of eqs. 6-9).

The library inverts each 6x6 chiral block by elimination without row
exchanges and refuses a build in which some block is not positive definite.
There is no global bound on kappa c_SW: the paper's own run of Sec. IV-D
(kappa 0.13310, c_SW 1.30255, so 6 kappa c_SW = 1.04) must build, and F, F^-1
and a solve must match the oracle; a c_SW that makes some blocks indefinite
must be refused, with the number of offending blocks equal to the number the
oracle's eigenvalues give.
"""
import os
import re
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

DIMS = (8, 8, 8, 16)
KAPPA_IVD, CSW_IVD = 0.13310, 1.30255


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def indefinite_blocks(F):
    """Number of (site, g5 sector) 6x6 blocks of the oracle's F whose smallest
    eigenvalue is not positive, and the smallest |eigenvalue| over all blocks."""
    w, v = np.linalg.eigh(oracle.gamma(4))
    M = F.reshape(-1, 12, 12)
    bad, closest = 0, np.inf
    for sel in (w > 0, w < 0):
        B = np.kron(v[:, sel], np.eye(3))
        ev = np.linalg.eigvalsh(np.einsum("ji,sjk,kl->sil", B.conj(), M, B))
        bad += int(np.count_nonzero(ev.min(axis=1) <= 0))
        closest = min(closest, float(np.abs(ev).min()))
    return bad, closest


def test_paper_run_parameters_build_and_solve():
    U = synth.random_links(DIMS, 0.3, 1071)
    lat = wc.Lattice(DIMS)
    lat.load_links(dev(U))
    lat.build_clover(KAPPA_IVD, CSW_IVD)
    say("6 kappa c_SW =", 6 * KAPPA_IVD * CSW_IVD)
    psi = synth.gaussian_source(DIMS, 2072)
    V = int(np.prod(DIMS))
    par = oracle.parity(DIMS).reshape(-1)
    eo_in = lat.pack(dev(psi), wc.FP64)
    for inverse in (0, 1):
        for p in (0, 1):
            eo_out = lat.new_eo(wc.FP64, 2)
            lat.apply_clover(lat.parity_view(eo_out, p, wc.FP64), lat.parity_view(eo_in, p, wc.FP64), p, inverse,
                             wc.FP64)
            out = lat.unpack(eo_out, wc.FP64).cpu().numpy().reshape(-1, 4, 3)
            sites = np.nonzero(par == p)[0]
            ref = oracle.clover_sites(U, KAPPA_IVD, CSW_IVD, psi, sites, bool(inverse))
            err, _ = site_errors(out[sites], ref, "F%s parity %d" % ("^-1" if inverse else "", p))
            assert err < 1e-13, (inverse, p)
    b = synth.gaussian_source(DIMS, 2071)
    for inner in (wc.FP32, wc.FP16):
        x, info = lat.solve(dev(b), KAPPA_IVD, CSW_IVD, 1e-10, inner_prec=inner)
        say(info)
        check_true_residual(U, KAPPA_IVD, CSW_IVD, b, x.cpu().numpy(), info, 1e-10)
    assert V == len(par)
    lat.close()


def test_indefinite_blocks_are_refused_and_counted():
    kappa, csw = 0.13, 5.0   # 6 kappa c_SW = 3.9: some blocks of these links turn indefinite
    U = synth.random_links(DIMS, 0.3, 1071)
    expect, closest = indefinite_blocks(oracle.clover_field(U, DIMS, kappa, csw))
    say("oracle: %d indefinite blocks; smallest |eigenvalue| %.3e" % (expect, closest))
    assert expect > 0 and closest > 1e-6
    lat = wc.Lattice(DIMS)
    lat.load_links(dev(U))
    with pytest.raises(wc.WCError) as e:
        lat.build_clover(kappa, csw)
    say(str(e.value))
    assert e.value.code == -1
    got = int(re.search(r"(\d+) of the (\d+) 6x6 clover blocks", str(e.value)).group(1))
    assert got == expect
    # no clover term is left behind: operators refuse, a solve asking for the
    # same parameters is refused the same way, and a good build recovers
    eo = lat.new_eo(wc.FP64, 1)
    with pytest.raises(wc.WCError) as e2:
        lat.apply_Dee_oo(lat.new_eo(wc.FP64, 1), eo, wc.FP64)
    assert e2.value.code == -4
    b = dev(synth.gaussian_source(DIMS, 2073))
    with pytest.raises(wc.WCError) as e3:
        lat.solve(b, kappa, csw, 1e-10)
    assert e3.value.code == -1
    x, info = lat.solve(b, 0.13, 1.0, 1e-10)
    check_true_residual(U, 0.13, 1.0, b.cpu().numpy(), x.cpu().numpy(), info, 1e-10)
    lat.close()
