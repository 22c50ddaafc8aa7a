"""The allocation-free D-hat_ee entry point against wc_apply_Dee_oo (same
kernels, so bit for bit), through the C ABI: two calls in a row on the same
GPU, the second on a smaller lattice, in FP64, FP32 and FP16; a lattice whose
intermediate field exceeds the fixed array is refused before any work."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_checks import say  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec", [wc.FP64, wc.FP32, wc.FP16])
def test_noalloc_matches_dhat_twice_second_smaller(prec):
    kappa = 0.13
    for dims, seed in (((8, 8, 8, 16), 1800), ((4, 6, 8, 10), 1801)):
        say("no-alloc D-hat", dims, prec)
        U = synth.random_links(dims, 0.3, seed)
        lat = wc.Lattice(dims)
        lat.load_links(dev(U))
        lat.build_clover(kappa, 1.0)
        psi = oracle.restrict(synth.gaussian_source(dims, seed + 100), 0)
        eo_in = lat.pack(dev(psi), prec)
        a = lat.new_eo(prec, 2)
        b = lat.new_eo(prec, 2)
        lat.apply_Dee_oo_noalloc(lat.parity_view(a, 0, prec), lat.parity_view(eo_in, 0, prec), prec)
        lat.apply_Dee_oo(lat.parity_view(b, 0, prec), lat.parity_view(eo_in, 0, prec), prec)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        lat.close()


def test_noalloc_refuses_a_field_larger_than_its_array():
    lib = wc.load_library()
    cap = lib.wc_noalloc_scratch_bytes()
    assert cap == 128 << 20
    dims = (32, 32, 32, 64)   # one FP64 parity: 192 MiB
    lat = wc.Lattice(dims)
    lat.load_links(synth.random_links_torch(dims, 0.3, 1802, device="cuda"))
    lat.build_clover(0.13, 1.0)
    assert lat.spinor_bytes(wc.FP64) > cap >= lat.spinor_bytes(wc.FP32)
    x = lat.new_eo(wc.FP64, 1)
    y = lat.new_eo(wc.FP64, 1)
    with pytest.raises(wc.WCError) as e:
        lat.apply_Dee_oo_noalloc(y, x, wc.FP64)
    assert e.value.code == -1 and "scratch" in str(e.value)
    lat.close()
