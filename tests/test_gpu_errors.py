"""Error paths of the C ABI on a GPU: every failure is reported through a
status code (and wc_last_error), never by a hang or a fault.  Conditions are
forced from the host (bad arguments, iteration caps, a non-finite source)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_not_ready_and_bad_enums():
    dims = (4, 4, 4, 4)
    lat = wc.Lattice(dims)
    b = dev(synth.gaussian_source(dims, 1))
    with pytest.raises(wc.WCError) as e:
        lat.solve(b, 0.12, 1.0, 1e-10)
    assert e.value.code == -4
    with pytest.raises(wc.WCError) as e:
        lat.apply_D(b, wc.FP64)
    assert e.value.code == -4
    lat.load_links(dev(synth.random_links(dims, 0.3, 2)))
    with pytest.raises(wc.WCError) as e:
        lat.apply_D(b, wc.FP64)         # clover not built yet
    assert e.value.code == -4
    lat.build_clover(0.12, 1.0)
    with pytest.raises(wc.WCError) as e:
        lat.apply_D(b, 7)
    assert e.value.code == -1
    for bad in ((-0.1, 1.0), (0.12, -1.0), (float("nan"), 1.0), (0.12, float("inf"))):
        with pytest.raises(wc.WCError) as e:
            lat.build_clover(*bad)      # kappa and c_SW must be finite and >= 0
        assert e.value.code == -1
    with pytest.raises(wc.WCError) as e:
        lat.solve(b, 0.12, 1.0, 0.0)
    assert e.value.code == -1
    with pytest.raises(wc.WCError) as e:
        lat.solve(b, 0.12, 1.0, 1e-10, inner_prec=9)
    assert e.value.code == -1


def test_nonfinite_source_rejected():
    dims = (4, 4, 4, 4)
    lat = wc.Lattice(dims)
    lat.load_links(dev(synth.random_links(dims, 0.3, 3)))
    b = synth.gaussian_source(dims, 4)
    b[1, 2, 3, 0, 2, 1] = np.nan
    with pytest.raises(wc.WCError) as e:
        lat.solve(dev(b), 0.12, 1.0, 1e-10)
    assert e.value.code == -1 and "non-finite" in str(e.value)


def test_iteration_caps_report_noconv():
    dims = (8, 8, 8, 8)
    lat = wc.Lattice(dims)
    lat.load_links(dev(synth.random_links(dims, 0.3, 5)))
    b = dev(synth.gaussian_source(dims, 6))
    x, info = lat.solve(b, 0.135, 1.0, 1e-12, inner_maxit=1, outer_maxit=1, raise_on_error=False)
    assert info["rc"] == -5 and info["status"] == -5
    assert 0 < info["true_rel_residual"] < 1 and torch.isfinite(x).all()
    x, info = lat.solve(b, 0.135, 1.0, 1e-12, inner_prec=wc.FP64, inner_maxit=3, raise_on_error=False)
    assert info["rc"] == -5
    assert torch.isfinite(x).all()


def test_past_critical_kappa_terminates():
    # kappa far past critical with c_SW = 0: the solver must stop within its caps
    dims = (4, 4, 4, 4)
    lat = wc.Lattice(dims)
    lat.load_links(dev(synth.unit_links(dims)))
    b = dev(synth.gaussian_source(dims, 7))
    x, info = lat.solve(b, 0.125, 0.0, 1e-10, inner_maxit=200, outer_maxit=5, raise_on_error=False)
    assert info["rc"] in (0, -5, -6)


def test_nonfinite_links_rejected():
    # a NaN entry must not slip through the load-time check (a maximum over the
    # entries drops NaN): the load is refused and the lattice has no links
    dims = (4, 4, 4, 4)
    lat = wc.Lattice(dims)
    U = synth.random_links(dims, 0.3, 5)
    lat.load_links(dev(U))
    U[2, 1, 0, 3, 2, 1, 1] = np.nan
    with pytest.raises(wc.WCError) as e:
        lat.load_links(dev(U))
    assert e.value.code == -1 and "non-finite" in str(e.value)
    b = dev(synth.gaussian_source(dims, 6))
    with pytest.raises(wc.WCError) as e:
        lat.solve(b, 0.12, 1.0, 1e-10)
    assert e.value.code == -4
    U[2, 1, 0, 3, 2, 1, 1] = np.inf
    with pytest.raises(wc.WCError) as e:
        lat.load_links(dev(U))
    assert e.value.code == -1
    lat.close()
