"""Argument checks of the Python binding, on the CPU.

The C ABI takes bare device pointers, so the binding checks every tensor it
hands over: canonical fields must be complex128 of the lattice's shape, and
even-odd (EO) buffers must hold at least the bytes the call touches (one
parity of wc_spinor_bytes, two for unpack).  A failed check raises ValueError
before any library call; a call with an invalid precision is passed on, for
the library to refuse.  Here the library is a stub that records its calls,
and tensors stay on the host (the device-pointer conversion is replaced), so
only the binding's own logic runs.
"""
import ctypes

import pytest

torch = pytest.importorskip("torch")

import paper_1709_08785_amd as wc  # noqa: E402

DIMS = (4, 4, 4, 4)
# one padded parity of 4^4 (128 sites, two 64-site tiles) per precision
SB = {wc.FP64: 128 * 192, wc.FP32: 128 * 96, wc.FP16: 128 * 52}


class StubLib:
    def __init__(self):
        self.calls = []

    def wc_spinor_bytes(self, h, prec):
        return SB.get(prec, 0)

    def __getattr__(self, name):
        def call(*args):
            self.calls.append(name)
            return 0
        return call


@pytest.fixture
def lat(monkeypatch):
    monkeypatch.setattr(wc, "_ptr", lambda t: ctypes.c_void_p(0))
    monkeypatch.setattr(wc.Lattice, "_sync_stream", lambda self: None)
    monkeypatch.setattr(wc, "load_library", lambda: StubLib())
    la = wc.Lattice.__new__(wc.Lattice)
    la.lib = StubLib()
    la.h = ctypes.c_void_p(1)
    la.dims = DIMS
    la.device = torch.device("cpu")
    la.volume = 256
    la.spinor_shape = (4, 4, 4, 4, 4, 3)
    la.link_shape = (4, 4, 4, 4, 4, 3, 3)
    yield la
    la.h = None


def eo(nbytes, dtype=torch.uint8):
    return torch.zeros(nbytes // torch.tensor([], dtype=dtype).element_size(), dtype=dtype)


@pytest.mark.parametrize("prec", [wc.FP64, wc.FP32, wc.FP16])
def test_eo_buffers_must_hold_one_parity(lat, prec):
    sb = SB[prec]
    lat.apply_mult(eo(sb), eo(sb), 0, prec)
    lat.apply_Dee_oo(eo(sb), eo(2 * sb), prec)  # a larger buffer is fine
    lat.apply_Dee_oo_noalloc(eo(sb), eo(sb), prec)
    lat.apply_clover(eo(sb), eo(sb), 1, True, prec)
    assert lat.lib.calls == ["wc_apply_mult", "wc_apply_Dee_oo", "wc_apply_Dee_oo_noalloc", "wc_apply_clover"]
    for call in (lambda: lat.apply_mult(eo(sb - 4), eo(sb), 0, prec),
                 lambda: lat.apply_mult(eo(sb), eo(sb - 4), 0, prec),
                 lambda: lat.apply_Dee_oo(eo(sb), eo(sb - 4), prec),
                 lambda: lat.apply_Dee_oo_noalloc(eo(sb - 4), eo(sb), prec),
                 lambda: lat.apply_clover(eo(sb), eo(sb // 2), 0, False, prec)):
        with pytest.raises(ValueError):
            call()
    assert len(lat.lib.calls) == 4


def test_eo_buffers_of_any_dtype_count_bytes(lat):
    sb = SB[wc.FP32]
    lat.apply_mult(eo(sb, torch.float32), eo(sb, torch.float64), 1, wc.FP32)
    with pytest.raises(ValueError):
        lat.apply_mult(eo(sb - 8, torch.float64), eo(sb), 1, wc.FP32)
    assert lat.lib.calls == ["wc_apply_mult"]


def test_invalid_precision_goes_to_the_library(lat):
    lat.apply_mult(eo(4), eo(4), 0, 7)
    assert lat.lib.calls == ["wc_apply_mult"]


def test_batches(lat):
    sb = SB[wc.FP16]
    outs = [eo(sb) for _ in range(3)]
    ins = [eo(sb) for _ in range(3)]
    lat.apply_mult_batch(outs, ins, 0, wc.FP16)
    lat.apply_Dee_oo_batch(outs, ins, wc.FP16)
    with pytest.raises(ValueError):
        lat.apply_mult_batch(outs, ins[:2], 0, wc.FP16)
    with pytest.raises(ValueError):
        lat.apply_Dee_oo_batch(outs[:2] + [eo(sb - 2)], ins, wc.FP16)
    assert lat.lib.calls == ["wc_apply_mult_batch", "wc_apply_Dee_oo_batch"]


def test_unpack_needs_both_parities(lat):
    sb = SB[wc.FP32]
    out = lat.unpack(eo(2 * sb), wc.FP32)
    assert out.dtype == torch.complex128 and tuple(out.shape) == lat.spinor_shape
    with pytest.raises(ValueError):
        lat.unpack(eo(sb), wc.FP32)
    assert lat.lib.calls == ["wc_unpack_spinor"]


def test_canonical_fields(lat):
    good = torch.zeros(lat.spinor_shape, dtype=torch.complex128)
    lat.pack(good, wc.FP32)
    lat.apply_D(good, wc.FP64)
    lat.load_links(torch.zeros(lat.link_shape, dtype=torch.complex128))
    lat.link_grad(good, good, 0.12, 1.0)
    assert lat.lib.calls == ["wc_pack_spinor", "wc_apply_D", "wc_load_links", "wc_link_grad"]
    bad = [torch.zeros(lat.spinor_shape, dtype=torch.complex64),
           torch.zeros((4, 4, 4, 4, 12), dtype=torch.complex128),
           torch.zeros((4, 4, 4, 8, 4, 3), dtype=torch.complex128)]
    for t in bad:
        for call in (lambda: lat.pack(t, wc.FP32), lambda: lat.apply_D(t, wc.FP64),
                     lambda: lat.link_grad(good, t, 0.12, 1.0), lambda: lat.link_grad(t, good, 0.12, 1.0)):
            with pytest.raises(ValueError):
                call()
    with pytest.raises(ValueError):
        lat.load_links(torch.zeros((4, 4, 4, 4, 4, 3, 2), dtype=torch.complex128))
    assert len(lat.lib.calls) == 4


def test_solves_check_sources_and_guess(lat):
    good = torch.zeros(lat.spinor_shape, dtype=torch.complex128)
    lat.solve(good, 0.12, 1.0, 1e-10)
    lat.solve(good, 0.12, 1.0, 1e-10, x0=good)
    lat.solve_batch([good, good], 0.12, 1.0, 1e-10)
    assert lat.lib.calls == ["wc_solve", "wc_solve", "wc_solve_batch"]
    wrong = torch.zeros((4, 4, 4, 8, 4, 3), dtype=torch.complex128)
    with pytest.raises(ValueError):
        lat.solve(wrong, 0.12, 1.0, 1e-10)
    with pytest.raises(ValueError):
        lat.solve(good, 0.12, 1.0, 1e-10, x0=wrong)
    with pytest.raises(ValueError):
        lat.solve_batch([good, wrong], 0.12, 1.0, 1e-10)
    assert len(lat.lib.calls) == 3


def test_solve_multi_checks_lengths_and_shapes(lat, monkeypatch):
    good = torch.zeros(lat.spinor_shape, dtype=torch.complex128)
    lib = StubLib()
    monkeypatch.setattr(wc, "load_library", lambda: lib)
    wc.solve_multi([lat, lat], [good, good], [0.12, 0.12], [1.0, 1.0], 1e-10)
    assert lib.calls == ["wc_solve_params_default", "wc_solve_multi"]
    with pytest.raises(ValueError):
        wc.solve_multi([lat, lat], [good], [0.12, 0.12], [1.0, 1.0], 1e-10)
    with pytest.raises(ValueError):
        wc.solve_multi([lat, lat], [good, good], [0.12], [1.0, 1.0], 1e-10)
    with pytest.raises(ValueError):
        wc.solve_multi([lat], [torch.zeros((2, 3), dtype=torch.complex128)], [0.12], [1.0], 1e-10)
    assert lib.calls == ["wc_solve_params_default", "wc_solve_multi"]
