"""Graph replay of the inner iteration chunk: every replay must reproduce the
eager launches exactly.  The chunk graph is replayed many times within a
solve (with host syncs and eager set-up work between replays) and across
solves from the cache; results and iteration counts are compared bit for bit
with the eager path, and against the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP16, wc.FP64])
def test_graph_equals_eager_single(inner):
    dims = (8, 8, 8, 8)
    kappa, csw = 0.12, 1.0
    print("graph single", inner, flush=True)
    U = synth.random_links(dims, 0.3, 1001)
    b = synth.gaussian_source(dims, 2001)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    bd = dev(b)
    x0, i0 = lat.solve(bd, kappa, csw, 1e-10, inner_prec=inner, use_graph=0, check_every=4)
    for rep in range(3):
        x1, i1 = lat.solve(bd, kappa, csw, 1e-10, inner_prec=inner, use_graph=1, check_every=4)
        assert torch.equal(x0, x1), rep
        assert i0["inner_iters_total"] == i1["inner_iters_total"] and i0["dslash_count"] == i1["dslash_count"]
    r, bn = oracle.residual(U, kappa, csw, b, x1.cpu().numpy())
    assert r / bn < 1e-10


def test_graph_equals_eager_uneven_batch():
    kappa, csw = 0.135, 1.0
    dims_list = [(4, 4, 4, 8), (8, 8, 8, 8), (6, 6, 6, 12)]
    print("graph multi", dims_list, flush=True)
    lats, bs = [], []
    for i, dims in enumerate(dims_list):
        lat = wc.Lattice(dims)
        lat.load_links(dev(synth.random_links(dims, 0.3, 1040 + i)))
        lats.append(lat)
        bs.append(dev(synth.gaussian_source(dims, 2040 + i)))
    xe, ie = wc.solve_multi(lats, bs, [kappa] * 3, [csw] * 3, 1e-10, use_graph=0)
    for rep in range(3):
        xg, ig = wc.solve_multi(lats, bs, [kappa] * 3, [csw] * 3, 1e-10, use_graph=1)
        for k in range(3):
            assert torch.equal(xe[k], xg[k]), (rep, k)
            assert ie[k]["inner_iters_total"] == ig[k]["inner_iters_total"]


def test_graph_cache_invalidated_by_new_clover():
    # the same lattice and buffers with a different kappa must not replay a stale graph
    dims = (8, 8, 8, 8)
    U = synth.random_links(dims, 0.3, 1050)
    b = synth.gaussian_source(dims, 2050)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    bd = dev(b)
    for kappa in (0.12, 0.13, 0.12):
        x, info = lat.solve(bd, kappa, 1.0, 1e-10, use_graph=1)
        r, bn = oracle.residual(U, kappa, 1.0, b, x.cpu().numpy())
        assert r / bn < 1e-10, kappa
