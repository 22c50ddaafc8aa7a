"""Batched solves on the GPU: several sources on one lattice (point sources,
the multi-RHS case) and lattices of different sizes in one set of launches.

Parity: every batched solution against the oracle's own solve at sizes the
oracle finishes in seconds (1e-10 relative), the oracle's true residual at the
full 32^3 x 64 size, and bit-identity with separate single solves (each
system keeps its own reductions in the same order).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_checks import check_true_residual, say  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def point_sources(dims):
    return [synth.point_source(dims, al, a) for al in range(4) for a in range(3)]


def test_batch_point_sources_small_vs_oracle():
    dims = (8, 8, 8, 8)
    kappa, csw = 0.135, 1.0
    say("batch 12 point sources", dims)
    U = synth.random_links(dims, 0.3, 1004)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    bs = point_sources(dims)
    xs, infos = lat.solve_batch([dev(b) for b in bs], kappa, csw, 1e-12)
    F = oracle.clover_field(U, dims, kappa, csw)
    for k in (0, 5, 11):
        x_ref, _, _ = oracle.solve(U, F, kappa, bs[k], tol=1e-13)
        assert rel(host(xs[k]), x_ref) < 1e-10, k
    for k, info in enumerate(infos):
        r, bn = oracle.residual(U, kappa, csw, bs[k], host(xs[k]))
        assert r / bn < 1e-12 and info["true_rel_residual"] < 1e-12, (k, info)


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP16, wc.FP64])
def test_batch_matches_single_solves(inner):
    dims = (8, 8, 8, 16)
    kappa, csw = 0.13, 1.0
    say("batch vs single", inner)
    U = synth.random_links(dims, 0.3, 1014)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    bs = [dev(synth.gaussian_source(dims, 2100 + k)) for k in range(3)]
    xs, infos = lat.solve_batch(bs, kappa, csw, 1e-10, inner_prec=inner)
    for k in range(3):
        x1, info1 = lat.solve(bs[k], kappa, csw, 1e-10, inner_prec=inner)
        d = float(torch.linalg.norm(x1 - xs[k]) / torch.linalg.norm(x1))
        assert d < 1e-9, (k, d)
        # the batched stencil rounds differently (another kernel, other FMA
        # contractions); at FP16 storage that moves the iteration count by a few
        assert abs(info1["inner_iters_total"] - infos[k]["inner_iters_total"]) <= max(2, 0.1 * info1["inner_iters_total"])
        assert infos[k]["true_rel_residual"] < 1e-10


@pytest.mark.parametrize("inner,recon", [(wc.FP32, 12), (wc.FP32, 8), (wc.FP16, 12)])
def test_batch_five_sources_two_groups(inner, recon):
    # five systems on one lattice whose sources differ in size, so that the
    # systems converge at different iterations and drop out of the batched
    # launches one by one
    dims = (8, 8, 8, 16)
    kappa, csw = 0.13, 1.0
    say("batch of 5", inner, recon)
    U = synth.random_links(dims, 0.3, 1015)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    lat.build_clover(kappa, csw)
    lat.set_link_recon(recon)
    bs = [dev(synth.gaussian_source(dims, 2200 + k) * (10.0 ** (k - 2))) for k in range(5)]
    bs[3] = dev(synth.point_source(dims, 1, 2))
    xs, infos = lat.solve_batch(bs, kappa, csw, 1e-10, inner_prec=inner)
    for k in range(5):
        r, bn = oracle.residual(U, kappa, csw, host(bs[k]), host(xs[k]))
        assert r / bn < 1e-10 and infos[k]["true_rel_residual"] < 1e-10, (k, infos[k])
        x1, info1 = lat.solve(bs[k], kappa, csw, 1e-10, inner_prec=inner)
        d = float(torch.linalg.norm(x1 - xs[k]) / torch.linalg.norm(x1))
        assert d < 1e-9, (k, d)


def test_multi_uneven_small_vs_oracle():
    kappa, csw = 0.135, 1.0
    dims_list = [(4, 4, 4, 4), (6, 6, 6, 12), (8, 8, 8, 16)]
    say("multi uneven", dims_list)
    lats, Us, bs = [], [], []
    for i, dims in enumerate(dims_list):
        U = synth.random_links(dims, 0.3, 1020 + i)
        lat = wc.Lattice(dims)
        lat.load_links(dev(U))
        lats.append(lat)
        Us.append(U)
        bs.append(synth.gaussian_source(dims, 2020 + i))
    xs, infos = wc.solve_multi(lats, [dev(b) for b in bs], [kappa] * 3, [csw] * 3, 1e-12)
    for i, dims in enumerate(dims_list):
        F = oracle.clover_field(Us[i], dims, kappa, csw)
        x_ref, _, _ = oracle.solve(Us[i], F, kappa, bs[i], tol=1e-13)
        assert rel(host(xs[i]), x_ref) < 1e-10, dims
        assert infos[i]["true_rel_residual"] < 1e-12


def test_multi_mixed_kappa_and_shared_lattice():
    # two systems on one lattice plus one on another, different kappa per lattice
    dims_a, dims_b = (8, 8, 8, 8), (4, 6, 8, 10)
    Ua, Ub = synth.random_links(dims_a, 0.3, 1031), synth.random_links(dims_b, 0.3, 1032)
    la, lb = wc.Lattice(dims_a), wc.Lattice(dims_b)
    la.load_links(dev(Ua))
    lb.load_links(dev(Ub))
    b = [synth.gaussian_source(dims_a, 2031), synth.gaussian_source(dims_b, 2032), synth.gaussian_source(dims_a, 2033)]
    xs, infos = wc.solve_multi([la, lb, la], [dev(v) for v in b], [0.12, 0.13, 0.12], [1.0, 1.0, 1.0], 1e-11)
    for k, (U, dims, kap) in enumerate([(Ua, dims_a, 0.12), (Ub, dims_b, 0.13), (Ua, dims_a, 0.12)]):
        check_true_residual(U, kap, 1.0, b[k], host(xs[k]), infos[k], 1e-11)


def test_multi_uneven_full_size_residual():
    # the uneven set the batch benchmark times (16^4 + 24^3x48 + 32^3x64, its
    # seeds): every system meets the oracle's true residual on its whole
    # lattice and agrees with its single solve to rounding
    kappa, csw = 0.135, 1.0
    dims_list = [(16, 16, 16, 16), (24, 24, 24, 48), (32, 32, 32, 64)]
    say("multi uneven full size", dims_list)
    lats, Us, bs = [], [], []
    for i, dims in enumerate(dims_list):
        U = synth.random_links(dims, 0.3, 1004 + 10 * i)
        lat = wc.Lattice(dims)
        lat.load_links(dev(U))
        lats.append(lat)
        Us.append(U)
        bs.append(synth.gaussian_source(dims, 2004 + 10 * i))
    xs, infos = wc.solve_multi(lats, [dev(b) for b in bs], [kappa] * 3, [csw] * 3, 1e-10)
    for i, dims in enumerate(dims_list):
        say(dims, infos[i])
        r, bn = oracle.residual(Us[i], kappa, csw, bs[i], host(xs[i]))
        say("oracle residual", dims, r / bn)
        assert r / bn < 1e-10, dims
        assert abs(r / bn - infos[i]["true_rel_residual"]) < 1e-12, dims
        x1, _ = lats[i].solve(dev(bs[i]), kappa, csw, 1e-10)
        assert rel(host(xs[i]), host(x1)) < 1e-9, dims
    for lat in lats:
        lat.close()
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_batch_full_size_point_sources_residual():
    # the 12 point sources on the 32^3 x 64 lattice, kappa 0.135: oracle true residual
    dims = (32, 32, 32, 64)
    kappa, csw = 0.135, 1.0
    say("batch 12 point sources", dims)
    U = synth.random_links(dims, 0.3, 1004)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    bs = point_sources(dims)
    xs, infos = lat.solve_batch([dev(b) for b in bs], kappa, csw, 1e-10)
    for k, info in enumerate(infos):
        say("point source", k, info)
        check_true_residual(U, kappa, csw, bs[k], host(xs[k]), info, 1e-10)


def test_multi_lattices_on_other_streams_with_new_kappa():
    # the second lattice's links are loaded on a stream of its own, and the batched
    # call asks for a kappa whose clover term is not built yet: the rebuild and the
    # earlier work on that stream must be ordered before the batch reads them
    dims_a, dims_b = (8, 8, 8, 8), (8, 8, 8, 16)
    Ua, Ub = synth.random_links(dims_a, 0.3, 1041), synth.random_links(dims_b, 0.3, 1042)
    other = torch.cuda.Stream()
    la = wc.Lattice(dims_a)
    la.load_links(dev(Ua))
    la.build_clover(0.12, 1.0)
    with torch.cuda.stream(other):
        lb = wc.Lattice(dims_b)
        lb.load_links(dev(Ub))
        lb.build_clover(0.12, 1.0)
    b = [synth.gaussian_source(dims_a, 2041), synth.gaussian_source(dims_b, 2042)]
    bd = [dev(v) for v in b]
    torch.cuda.synchronize()
    xs, infos = wc.solve_multi([la, lb], bd, [0.13, 0.135], [1.0, 1.0], 1e-11)
    for k, (U, kap) in enumerate([(Ua, 0.13), (Ub, 0.135)]):
        check_true_residual(U, kap, 1.0, b[k], host(xs[k]), infos[k], 1e-11)
    la.close()
    lb.close()


def test_multi_after_destroying_and_recreating_a_lattice():
    # a cached batch names its lattices by serial number: a lattice destroyed and
    # created again (often at the same address) with other links must not reuse
    # the graphs recorded with the old one's buffers
    dims = (8, 8, 8, 8)
    kappa, csw = 0.13, 1.0
    la = wc.Lattice(dims)
    Ua = synth.random_links(dims, 0.3, 1051)
    la.load_links(dev(Ua))
    bs = [synth.gaussian_source(dims, 2051), synth.gaussian_source(dims, 2052)]
    for round_ in range(3):
        Ub = synth.random_links(dims, 0.3, 1060 + round_)
        lb = wc.Lattice(dims)
        lb.load_links(dev(Ub))
        xs, infos = wc.solve_multi([la, lb], [dev(v) for v in bs], [kappa] * 2, [csw] * 2, 1e-11)
        say("round", round_, [i["true_rel_residual"] for i in infos])
        check_true_residual(Ua, kappa, csw, bs[0], host(xs[0]), infos[0], 1e-11)
        check_true_residual(Ub, kappa, csw, bs[1], host(xs[1]), infos[1], 1e-11)
        lb.close()
    la.close()
