"""Kernel accounting under HIP-event timing: the inner loop queues several
iterations between convergence reads, and launches queued after a system
stopped return at once.  Those launches must not count as work: the stencil
launches recorded for a solve are then exactly the iterations done (two
MULTs per D-hat, two D-hats per iteration, one fewer at a half-step exit),
and their bytes are the per-launch algorithmic bytes times that count."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU but never run there
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("inner,name", [(wc.FP32, "fp32"), (wc.FP16, "fp16")])
def test_timed_launches_match_iterations(inner, name):
    dims = (8, 8, 8, 16)
    U = synth.random_links(dims, 0.3, 1016)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    b = dev(synth.gaussian_source(dims, 2016))
    x, info0 = lat.solve(b, 0.13, 1.0, 1e-10, inner_prec=inner)
    lat.reset_kernel_stats()
    lat.set_timing(True)
    x, info = lat.solve(b, 0.13, 1.0, 1e-10, inner_prec=inner)
    lat.set_timing(False)
    st = lat.kernel_stats()
    print(info, {k: v["launches"] for k, v in st.items()}, flush=True)
    sys.stdout.flush()
    assert info["inner_iters_total"] == info0["inner_iters_total"]
    hop, dh = st["mult_hopinv_" + name], st["mult_dhat_" + name]
    its, calls = info["inner_iters_total"], info["inner_calls"]
    # one first-half MULT per D-hat; a half-step exit skips the second D-hat
    assert hop["launches"] == dh["launches"]
    assert 2 * its - calls <= dh["launches"] <= 2 * its
    # every counted launch carries the same algorithmic bytes
    per = {k: v["bytes"] / v["launches"] for k, v in (("h", hop), ("d", dh))}
    assert per["h"] > 0 and per["d"] > 0
