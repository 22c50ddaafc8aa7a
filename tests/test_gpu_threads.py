"""Two host threads, each with its own lattice and its own HIP stream, solve
at the same time: lattice handles share no state (errors are per thread,
graphs are recorded in thread-local capture mode on each lattice's private
stream), so every solution must equal, bit for bit, the same solve run
alone, and pass the oracle's residual."""
import sys
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU but never run there
    pytest.skip("no GPU", allow_module_level=True)

import paper_1709_08785_amd as wc  # noqa: E402

FORMS = [dict(), dict(inner_prec=wc.FP16), dict(outer="dc")]


def case(k):
    dims = (8, 8, 8, 16) if k == 0 else (6, 6, 6, 10)
    return dims, synth.random_links(dims, 0.3, 1120 + k), synth.gaussian_source(dims, 2120 + k)


def run_case(k, out, errors):
    try:
        dims, U, b = case(k)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            lat = wc.Lattice(dims)
            lat.set_block_size(256)
            lat.load_links(torch.from_numpy(U).cuda())
            bd = torch.from_numpy(b).cuda()
            xs = []
            for rep in range(3):
                for kw in FORMS:
                    x, info = lat.solve(bd, 0.13, 1.0, 1e-10, **kw)
                    xs.append(x.clone())
            stream.synchronize()
            out[k] = [x.cpu().numpy() for x in xs]
            lat.close()
    except Exception as e:  # reported by the main thread
        errors.append((k, repr(e)))


def test_two_threads_solve_concurrently():
    print("two threads", flush=True)
    sys.stdout.flush()
    out, errors = {}, []
    threads = [threading.Thread(target=run_case, args=(k, out, errors)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=240)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    # the same solves alone, one thread
    for k in range(2):
        alone = {}
        run_case(k, alone, errors)
        assert not errors, errors
        dims, U, b = case(k)
        for i, (xc, xa) in enumerate(zip(out[k], alone[k])):
            assert np.array_equal(xc, xa), (k, i)
            r, bn = oracle.residual(U, 0.13, 1.0, b, xc)
            assert r / bn < 1e-10, (k, i)


def test_one_lattice_on_alternating_streams():
    # the binding rebinds the lattice to torch's current stream on every call;
    # graphs recorded while one stream was current replay on the other
    dims, U, b = case(0)
    lat = wc.Lattice(dims)
    lat.load_links(torch.from_numpy(U).cuda())
    bd = torch.from_numpy(b).cuda()
    x0, _ = lat.solve(bd, 0.13, 1.0, 1e-10)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(2):
        for s in (s1, s2):
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                x, info = lat.solve(bd, 0.13, 1.0, 1e-10)
                s.synchronize()
            assert torch.equal(x, x0), rep
    lat.close()
