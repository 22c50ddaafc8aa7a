"""GPU parity of the solver's launch shape: the stencil and vector kernels at
64, 128 and 256 threads per block (1, 2 or 4 tiles of 64 sites), pinned with
wc_set_block_size or chosen by the tuner.  Every size must reproduce the
oracle's operator and solution; only the rounding order of the reductions may
change.  The 6x6x6x10 lattice has 1080 sites per parity, so the last block is
partial at every size."""
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

RAGGED = (6, 6, 6, 10)
TOL = {wc.FP64: 1e-13, wc.FP32: 1e-5, wc.FP16: 2e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def lattice(dims, seed, kappa=None, csw=1.0):
    U = synth.random_links(dims, 0.3, seed)
    lat = wc.Lattice(dims)
    lat.load_links(dev(U))
    if kappa is not None:
        lat.build_clover(kappa, csw)
    return lat, U


@pytest.mark.parametrize("prec", [wc.FP64, wc.FP32, wc.FP16])
@pytest.mark.parametrize("bs", [64, 128, 256])
def test_dhat_each_block_size(bs, prec):
    say("dhat, block size", bs, prec)
    kappa = 0.13
    lat, U = lattice(RAGGED, 1060, kappa)
    lat.set_block_size(bs)
    Finv = oracle.site_invert(oracle.clover_field(U, RAGGED, kappa, 1.0))
    psi = oracle.restrict(synth.gaussian_source(RAGGED, 2060), 0)
    eo_in = lat.pack(dev(psi), prec)
    eo_out = lat.new_eo(prec, 2)
    lat.apply_Dee_oo(lat.parity_view(eo_out, 0, prec), lat.parity_view(eo_in, 0, prec), prec)
    out = host(lat.unpack(eo_out, prec))
    assert rel(out, oracle.dhat_ee(U, Finv, kappa, psi)) < TOL[prec]
    lat.close()


@pytest.mark.parametrize("inner", [wc.FP32, wc.FP16, wc.FP64])
@pytest.mark.parametrize("bs", [64, 128, 256])
def test_solve_each_block_size_matches_oracle(bs, inner):
    say("solve, block size", bs, inner)
    kappa = 0.13
    lat, U = lattice(RAGGED, 1061)
    lat.set_block_size(bs)
    b = synth.gaussian_source(RAGGED, 2061)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12, inner_prec=inner)
    say(info)
    assert info["block_size"] == bs
    r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
    assert r / bn < 1e-12
    F = oracle.clover_field(U, RAGGED, kappa, 1.0)
    x_ref, _, _ = oracle.solve(U, F, kappa, b, tol=1e-13)
    assert rel(host(x), x_ref) < 1e-10
    lat.close()


def test_block_sizes_agree_to_rounding():
    # the same system at every size: the solutions differ by the rounding of
    # the reductions only, and the iteration counts stay within a couple
    dims, kappa = (8, 8, 8, 16), 0.1355
    lat, U = lattice(dims, 1062)
    b = dev(synth.gaussian_source(dims, 2062))
    xs, its = {}, {}
    for bs in (64, 128, 256):
        lat.set_block_size(bs)
        x, info = lat.solve(b, kappa, 1.0, 1e-12)
        xs[bs], its[bs] = host(x), info["inner_iters_total"]
    say(its)
    for bs in (64, 128):
        assert rel(xs[bs], xs[256]) < 1e-10
        assert abs(its[bs] - its[256]) <= max(2, 0.05 * its[256])
    lat.close()


def test_graph_replay_bit_exact_at_block_size_64():
    dims, kappa = (8, 8, 8, 8), 0.12
    lat, U = lattice(dims, 1063)
    lat.set_block_size(64)
    b = dev(synth.gaussian_source(dims, 2063))
    x0, i0 = lat.solve(b, kappa, 1.0, 1e-10, use_graph=0, check_every=4)
    for rep in range(2):
        x1, i1 = lat.solve(b, kappa, 1.0, 1e-10, use_graph=1, check_every=4)
        assert torch.equal(x0, x1), rep
        assert i0["inner_iters_total"] == i1["inner_iters_total"]
    lat.close()


def test_batch_at_block_size_64_matches_single_solves():
    dims, kappa = (8, 8, 8, 8), 0.12
    lat, U = lattice(dims, 1064)
    lat.set_block_size(64)
    bs_ = [dev(synth.gaussian_source(dims, 2064 + k)) for k in range(3)]
    xb, infos = lat.solve_batch(bs_, kappa, 1.0, 1e-10)
    for k in range(3):
        assert infos[k]["block_size"] == 64
        x1, _ = lat.solve(bs_[k], kappa, 1.0, 1e-10)
        assert rel(host(xb[k]), host(x1)) < 1e-9
        r, bn = oracle.residual(U, kappa, 1.0, host(bs_[k]), host(xb[k]))
        assert r / bn < 1e-10
    lat.close()


def test_uneven_batch_takes_the_largest_lattice_block_size():
    kappa = 0.13
    dims_list = [(4, 4, 4, 8), (8, 8, 8, 8), (6, 6, 6, 10)]
    pins = [64, 128, 256]
    lats, Us, bs_ = [], [], []
    for i, (dims, pin) in enumerate(zip(dims_list, pins)):
        lat, U = lattice(dims, 1065 + i)
        lat.set_block_size(pin)
        lats.append(lat)
        Us.append(U)
        bs_.append(dev(synth.gaussian_source(dims, 2065 + i)))
    xs, infos = wc.solve_multi(lats, bs_, [kappa] * 3, [1.0] * 3, 1e-10)
    for k in range(3):
        assert infos[k]["block_size"] == 128  # 8^4 has the most sites
        r, bn = oracle.residual(Us[k], kappa, 1.0, host(bs_[k]), host(xs[k]))
        assert r / bn < 1e-10
    for lat in lats:
        lat.close()


def test_tuner_reports_timings_and_applies_its_choice():
    dims, kappa = (16, 16, 16, 16), 0.13
    lat, U = lattice(dims, 1068, kappa)
    assert lat.block_size(wc.FP32) == 0  # not tuned yet
    res = lat.tune_block_size(wc.FP32)
    say(res)
    us = res["us_per_pair"]
    assert all(v > 0 for v in us.values())
    # the rule: starting from 256 threads at chunk 32, a shape replaces the
    # best so far only when 3% faster; so the chosen block size is within 3%
    # of the fastest one at the chosen chunk
    assert res["threads"] == lat.block_size(wc.FP32)
    assert res["chunk"] == lat.xcd_chunk(wc.FP32) and res["chunk"] in (8, 16, 32, 64)
    assert us[res["threads"]] <= min(us.values()) / 0.97 + 1e-9
    best = res["threads"]
    b = synth.gaussian_source(dims, 2068)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-10)
    assert info["block_size"] == best
    r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
    assert r / bn < 1e-10
    lat.close()


def test_first_solve_tunes_and_pin_overrides():
    dims, kappa = (8, 8, 8, 8), 0.12
    lat, U = lattice(dims, 1069)
    b = dev(synth.gaussian_source(dims, 2069))
    assert lat.block_size(wc.FP16) == 0
    x, info = lat.solve(b, kappa, 1.0, 1e-10, inner_prec=wc.FP16)
    assert info["block_size"] in (64, 128, 256)
    assert lat.block_size(wc.FP16) == info["block_size"]
    lat.set_block_size(128)
    x, info = lat.solve(b, kappa, 1.0, 1e-10, inner_prec=wc.FP16)
    assert info["block_size"] == 128 == lat.block_size(wc.FP32)
    with pytest.raises(wc.WCError):
        lat.set_block_size(96)
    lat.set_block_size(0)
    assert lat.block_size(wc.FP16) in (64, 128, 256)
    lat.close()


@pytest.mark.parametrize("recon", [8, 18])
@pytest.mark.parametrize("bs", [64, 128])
def test_small_blocks_with_other_link_forms(bs, recon):
    dims, kappa = RAGGED, 0.13
    say("block size", bs, "link form", recon)
    lat, U = lattice(dims, 1071)
    lat.set_link_recon(recon)
    lat.set_block_size(bs)
    b = synth.gaussian_source(dims, 2071)
    x, info = lat.solve(dev(b), kappa, 1.0, 1e-12)
    assert info["block_size"] == bs
    r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
    assert r / bn < 1e-12
    lat.close()


def test_tuner_cache_file(tmp_path):
    # a tuned shape is written to the cache file and taken from it by the next
    # lattice of the same case, without timing (the stored microseconds come back)
    dims, kappa = (8, 8, 8, 16), 0.13
    path = tmp_path / "tune.txt"
    wc.set_tune_cache(str(path))
    try:
        lat, U = lattice(dims, 1070, kappa)
        r1 = lat.tune_block_size(wc.FP16)
        lines = path.read_text().splitlines()
        say(lines)
        assert len(lines) == 1 and lines[0].startswith("wc-tune-v3 ")
        f = lines[0].split()
        # wc-tune-v3 arch CUs Lx Ly Lz Lt prec recon pinned-cap threads chunk cap-mult cap-dhat us64 us128 us256
        assert [int(v) for v in f[3:7]] == list(dims) and int(f[7]) == wc.FP16 and int(f[8]) == 12
        assert int(f[9]) == -1
        assert int(f[10]) == r1["threads"] and int(f[11]) == r1["chunk"]
        assert int(f[12]) == r1["wave_cap"]["mult"] and int(f[13]) == r1["wave_cap"]["dhat"]
        lat2, _ = lattice(dims, 1070, kappa)
        r2 = lat2.tune_block_size(wc.FP16)
        assert r2["threads"] == r1["threads"] and r2["chunk"] == r1["chunk"] and r2["wave_cap"] == r1["wave_cap"]
        assert all(abs(r2["us_per_pair"][k] - round(r1["us_per_pair"][k], 3)) < 1e-9 for k in (64, 128, 256))
        assert len(path.read_text().splitlines()) == 1
        lat.close()
        lat2.close()
    finally:
        wc.set_tune_cache(None)


def test_tuner_cache_bypassed_under_a_pinned_shape(tmp_path):
    # a tuning under a pinned block size or chunk neither writes the cache file
    # nor takes a stored shape from it
    dims, kappa = (8, 8, 8, 16), 0.13
    path = tmp_path / "tune.txt"
    wc.set_tune_cache(str(path))
    lat, U = lattice(dims, 1072, kappa)
    try:
        lat.set_block_size(64)
        r0 = lat.tune_block_size(wc.FP32)
        assert r0["threads"] == 64
        assert not path.exists() or path.read_text() == ""
        lat.set_block_size(0)
        r1 = lat.tune_block_size(wc.FP32)
        assert len(path.read_text().splitlines()) == 1
        other = 128 if r1["threads"] != 128 else 64
        lat.set_block_size(other)
        r2 = lat.tune_block_size(wc.FP32)
        say(r1, r2)
        assert r2["threads"] == other and lat.block_size(wc.FP32) == other
        lat.set_block_size(0)
        lat.set_xcd_chunk(16)
        r3 = lat.tune_block_size(wc.FP32)
        assert r3["chunk"] == 16
        assert len(path.read_text().splitlines()) == 1
    finally:
        lat.set_block_size(0)
        lat.set_xcd_chunk(-1)
        lat.close()
        wc.set_tune_cache(None)


def test_tuner_with_a_pinned_block_size_chooses_for_that_size():
    dims, kappa = (16, 16, 16, 16), 0.13
    lat, U = lattice(dims, 1071, kappa)
    lat.set_block_size(64)
    try:
        res = lat.tune_block_size(wc.FP32)
        say(res)
        assert res["threads"] == 64 and lat.block_size(wc.FP32) == 64
        assert res["chunk"] in (8, 16, 32, 64)
        assert all(v in (0, 8, 12) for v in res["wave_cap"].values())
        b = synth.gaussian_source(dims, 2071)
        x, info = lat.solve(dev(b), kappa, 1.0, 1e-10)
        assert info["block_size"] == 64
        r, bn = oracle.residual(U, kappa, 1.0, b, host(x))
        assert r / bn < 1e-10
    finally:
        lat.set_block_size(0)
        lat.close()
