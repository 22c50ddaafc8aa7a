"""GPU parity of the full FP32 link form (wc_set_link_recon 18) and of the
handling of links that are not SU(3).

Two-column storage rebuilds the third column as conj(col0 x col1), exact only
for special-unitary links (Sec. III-A).  Links pushed off SU(3) by a small
random non-unitary term must be detected when loaded, switch the FP32 stencil
to full links, refuse the two-column forms and FP16, and still give the
oracle's operator and solution; SU(3) links loaded afterwards return the
lattice to the default form."""
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


def off_su3(U, size, seed):
    """U + size * G with G a complex Gaussian 3x3 per link: not unitary."""
    g = synth.rng(seed)
    G = g.standard_normal(U.shape + (2,))
    return U + size * (G[..., 0] + 1j * G[..., 1])


def test_full_links_on_su3_match_oracle_and_recon12():
    dims, kappa = (6, 6, 6, 10), 0.13
    U = synth.random_links(dims, 0.3, 1095)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    lat.build_clover(kappa, 1.0)
    assert lat.link_recon == 12 and lat.link_su3_error < 1e-12
    psi = synth.gaussian_source(dims, 2095)
    y12 = host(lat.apply_D(dev(psi), wc.FP32))
    lat.set_link_recon(18)
    assert lat.link_recon == 18
    y18 = host(lat.apply_D(dev(psi), wc.FP32))
    ref = oracle.apply_D(U, oracle.clover_field(U, dims, kappa, 1.0), kappa, psi)
    say("recon 18", rel(y18, ref), "recon 12", rel(y12, ref))
    assert rel(y18, ref) < 1e-6 and rel(y12, ref) < 1e-5
    b = synth.gaussian_source(dims, 2096)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12)
    r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
    assert r / bn < 1e-12
    lat.close()


def test_links_off_su3_switch_to_full_links():
    dims, kappa = (6, 6, 6, 10), 0.13
    U = off_su3(synth.random_links(dims, 0.3, 1097), 0.02, 3097)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    say("su3 error", lat.link_su3_error)
    assert lat.link_su3_error > 1e-3
    assert lat.link_recon == 18  # chosen on load
    for form in (12, 8):
        with pytest.raises(wc.WCError) as e:
            lat.set_link_recon(form)
        assert e.value.code == -1
    assert lat.link_recon == 18
    lat.build_clover(kappa, 1.0)
    F = oracle.clover_field(U, dims, kappa, 1.0)
    psi = synth.gaussian_source(dims, 2097)
    for prec, tol in ((wc.FP64, 1e-13), (wc.FP32, 1e-6)):
        y = host(lat.apply_D(dev(psi), prec))
        assert rel(y, oracle.apply_D(U, F, kappa, psi)) < tol, prec
    # the FP32 inner solve on full links converges like on SU(3) links; FP16 is refused
    b = synth.gaussian_source(dims, 2098)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12)
    say(info)
    x_ref, _, _ = oracle.solve(U, F, kappa, b, tol=1e-13)
    assert rel(host(x), x_ref) < 1e-10
    assert info["outer_iters"] <= 2
    with pytest.raises(wc.WCError) as e:
        lat.solve(dev(b), kappa, 1.0, 1e-10, inner_prec=wc.FP16)
    assert e.value.code == -1 and "SU(3)" in str(e.value)
    # SU(3) links again: back to the default two-column form, FP16 allowed
    U2 = synth.random_links(dims, 0.3, 1098)
    lat.load_links(dev(U2))
    assert lat.link_recon == 12 and lat.link_su3_error < 1e-12
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-10, inner_prec=wc.FP16)
    r, bn = oracle.residual(U2, kappa, 1.0, b, host(x))
    assert r / bn < 1e-10
    lat.close()


def test_chosen_full_form_survives_reload():
    dims = (4, 4, 4, 8)
    lat = wc.Lattice(dims)
    lat.load_links(dev(synth.random_links(dims, 0.3, 1099)))
    lat.set_link_recon(18)
    lat.load_links(dev(synth.random_links(dims, 0.3, 1100)))
    assert lat.link_recon == 18  # the caller's choice, not the automatic one
    lat.close()


def test_callers_form_restored_after_links_off_su3():
    dims = (4, 4, 4, 8)
    U = synth.random_links(dims, 0.3, 1101)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    lat.set_link_recon(8)
    lat.load_links(dev(off_su3(U, 0.02, 3101)))
    assert lat.link_recon == 18
    lat.load_links(dev(U))
    assert lat.link_recon == 8
    lat.close()


def test_full_links_in_one_launch_loop_and_batches():
    # links off SU(3) (so the lattice reads them in full) through the
    # one-launch inner loop and a batched solve, both against the oracle
    dims, kappa = (8, 8, 8, 8), 0.12
    U = off_su3(synth.random_links(dims, 0.3, 1102), 0.02, 3102)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    assert lat.link_recon == 18
    F = oracle.clover_field(U, dims, kappa, 1.0)
    b = synth.gaussian_source(dims, 2102)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12, persistent=1)
    say(info)
    assert info["persistent_calls"] == info["inner_calls"] > 0
    x_ref, _, _ = oracle.solve(U, F, kappa, b, tol=1e-13)
    assert rel(host(x), x_ref) < 1e-10
    bs = [dev(synth.gaussian_source(dims, 2103 + k)) for k in range(3)]
    xs, infos = lat.solve_batch(bs, kappa, 1.0, 1e-10)
    for k in range(3):
        r, bn = oracle.residual(U, kappa, 1.0, host(bs[k]), host(xs[k]))
        assert r / bn < 1e-10, k
    # a batch over lattices with different link forms is refused
    lat2 = wc.Lattice(dims)
    lat2.load_links(dev(synth.random_links(dims, 0.3, 1103)))
    assert lat2.link_recon == 12
    with pytest.raises(wc.WCError) as e:
        wc.solve_multi([lat, lat2], [bs[0], bs[1]], [kappa] * 2, [1.0] * 2, 1e-10)
    assert e.value.code == -1
    lat.close()
    lat2.close()
