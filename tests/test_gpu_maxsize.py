"""The largest lattice of the test-suite, 64^3x128 (16.8M sites per parity,
about 150 GB of device memory in use).  Its FP64 clover slabs are 9.7 GB and
its spinor slabs 3.2 GB, so a byte offset held in 32 bits anywhere on the path
would show.  The operator is checked on sampled output sites against the
oracle's site-by-site D, and the FP16-inner solve by the oracle's FP64 true
residual over the whole lattice."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU but never run there
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402

DIMS = (64, 64, 64, 128)
KAPPA, CSW = 0.1355, 1.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big():
    say("links 64^3x128")
    Ud = synth.random_links_torch(DIMS, 0.3, 1090, device="cuda")
    lat = wc.Lattice(DIMS)
    lat.load_links(Ud)
    U = Ud.cpu().numpy()
    del Ud
    torch.cuda.empty_cache()
    lat.build_clover(KAPPA, CSW)
    say("lattice ready")
    yield lat, U
    lat.close()


def test_apply_D_sampled_sites_64x64x64x128(big):
    lat, U = big
    psi = synth.gaussian_source(DIMS, 2090)
    say("apply_D FP32")
    out = lat.apply_D(torch.from_numpy(psi).cuda(), wc.FP32).cpu().numpy().reshape(-1, 4, 3)
    V = int(np.prod(DIMS))
    g = synth.rng(11)
    # random sites plus both ends of the site order and of each parity slab
    sites = np.concatenate([g.integers(0, V, 3000), [0, 1, V // 2 - 1, V // 2, V - 2, V - 1]])
    ref = oracle.apply_D_sites(U, KAPPA, CSW, psi, sites)
    err = np.linalg.norm(out[sites] - ref) / np.linalg.norm(ref)
    say("rel err", err)
    assert err < 1e-5


def test_solve_64x64x64x128_fp16_oracle_residual(big):
    lat, U = big
    b = synth.z2_source(DIMS, 2091)
    say("solve FP16 inner")
    x, info = lat.solve(torch.from_numpy(b).cuda(), KAPPA, CSW, 1e-10, inner_prec=wc.FP16)
    say(info)
    xh = x.cpu().numpy()
    del x
    say("oracle residual")
    r, bn = oracle.residual(U, KAPPA, CSW, b, xh)
    say("oracle", r / bn)
    assert r / bn < 1e-10
    assert abs(r / bn - info["true_rel_residual"]) < 1e-12
