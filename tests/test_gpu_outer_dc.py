"""GPU parity of the defect-correction outer iteration (the variant of the
outer loop beside the flexible BiCGStab of Algorithm 1): x_e += M r_e with
r_e recomputed in FP64 after every inner solve.  The solution is the unique
solution of D x = b, so it is checked against the oracle's solve (1e-10
relative) and against the oracle's FP64 residual of the returned x.
"""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


_lat = {}


def lattice(dims, seed, kappa):
    key = (dims, seed, kappa)
    if key not in _lat:
        U = synth.random_links(dims, 0.3, seed)
        lat = wc.Lattice(dims)
        lat.load_links(dev(U))
        lat.build_clover(kappa, 1.0)
        _lat[key] = (lat, U)
    return _lat[key]


@pytest.mark.parametrize("inner,recon", [(wc.FP32, 12), (wc.FP32, 8), (wc.FP16, 12)])
def test_dc_solve_matches_oracle(inner, recon):
    dims, kappa = (8, 8, 8, 8), 0.12
    say("dc solve", inner, recon)
    lat, U = lattice(dims, 1001, kappa)
    lat.set_link_recon(recon)
    b = synth.gaussian_source(dims, 2001)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    x_ref, _, _ = oracle.solve(U, F, kappa, b, tol=1e-13)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12, inner_prec=inner, outer="dc")
    lat.set_link_recon(12)
    say(info)
    r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
    assert r / bn < 1e-12 and info["true_rel_residual"] < 1e-12
    assert rel(host(x), x_ref) < 1e-10
    # one inner call per outer step
    assert info["inner_calls"] == info["outer_iters"]


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP16])
def test_dc_near_critical_kappa(inner):
    dims, kappa = (8, 8, 8, 16), 0.1355
    lat, U = lattice(dims, 1002, kappa)
    b = synth.gaussian_source(dims, 2002)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-10, inner_prec=inner, outer="dc")
    say(info)
    r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
    assert r / bn < 1e-10


def test_dc_iteration_cap_reports_no_convergence():
    dims, kappa = (8, 8, 8, 8), 0.12
    lat, U = lattice(dims, 1001, kappa)
    b = synth.gaussian_source(dims, 2003)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12, inner_prec=wc.FP16, outer="dc", outer_maxit=1,
                        raise_on_error=False)
    assert info["rc"] == -5 and info["status"] == -5
    assert info["true_rel_residual"] > 1e-12
    # the iterate it leaves is the one-step correction: its residual is near the inner tolerance
    assert info["true_rel_residual"] < 1e-2


def test_dc_batch_of_sources():
    dims, kappa = (8, 8, 8, 16), 0.13
    lat, U = lattice(dims, 1014, kappa)
    bs = [synth.gaussian_source(dims, 2300 + k) for k in range(3)]
    xs, infos = lat.solve_batch([dev(b) for b in bs], kappa, 1.0, 1e-10, outer="dc")
    for k in range(3):
        r, bn = oracle.residual(U, kappa, 1.0, bs[k], host(xs[k]))
        assert r / bn < 1e-10, (k, infos[k])


def test_dc_bad_outer_value_rejected():
    dims, kappa = (4, 4, 4, 4), 0.12
    lat, U = lattice(dims, 1003, kappa)
    with pytest.raises(wc.WCError) as e:
        lat.solve(dev(synth.gaussian_source(dims, 1)), kappa, 1.0, 1e-10, outer=7)
    assert e.value.code == -1
