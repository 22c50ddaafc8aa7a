"""The C ABI on its own: a C program (tests/c_client/wc_solve_file.c, built
with gcc by the build step) loads links and a source through wc.h and the HIP
runtime only, in a process without Python or torch, and solves; its solution
is checked against the FP64 oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU but never run there
    pytest.skip("no GPU", allow_module_level=True)

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "wc_solve_file")


def test_c_client_solves_through_the_abi(tmp_path):
    if not os.path.exists(BIN):
        pytest.skip("the C client is not built (run __graft_entry__.build())")
    dims, kappa, csw = (6, 6, 6, 10), 0.13, 1.0
    U = synth.random_links(dims, 0.3, 1110)
    b = synth.gaussian_source(dims, 2110)
    np.ascontiguousarray(U, dtype=np.complex128).tofile(tmp_path / "links.bin")
    np.ascontiguousarray(b, dtype=np.complex128).tofile(tmp_path / "b.bin")
    args = [BIN] + [str(d) for d in dims] + [repr(kappa), repr(csw), "1e-11",
                                             str(tmp_path / "links.bin"), str(tmp_path / "b.bin"),
                                             str(tmp_path / "x.bin")]
    print("running", " ".join(args), flush=True)
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    sys.stdout.flush()
    assert r.returncode == 0, r.stderr
    fields = r.stdout.split()
    assert fields[0] == "status" and int(fields[1]) == 0
    x = np.fromfile(tmp_path / "x.bin", dtype=np.complex128).reshape(b.shape)
    rr, bn = oracle.residual(U, kappa, csw, b, x)
    assert rr / bn < 1e-11
    assert abs(rr / bn - float(fields[7])) < 1e-12
    x_ref, _, _ = oracle.solve(U, oracle.clover_field(U, dims, kappa, csw), kappa, b, tol=1e-13)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-9
