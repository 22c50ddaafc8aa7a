"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wc.h")
LIB = os.path.join(ROOT, "paper_1709_08785_amd", "libwc.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wc_[A-Za-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_1709_08785_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["wc_create_lattice", "wc_load_links", "wc_build_clover", "wc_apply_D", "wc_apply_Dee_oo",
                 "wc_solve", "wc_destroy_lattice", "wc_last_error"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_create_rejects_bad_extents_before_gpu(lib):
    lib.wc_create_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.wc_last_error.restype = ctypes.c_char_p
    for dims in [(4, 4, 4, 5), (0, 4, 4, 4), (4, 4, 4, 1), (-2, 4, 4, 4)]:
        h = ctypes.c_void_p()
        rc = lib.wc_create_lattice((ctypes.c_int * 4)(*dims), None, ctypes.byref(h))
        assert rc == -1 and not h.value
        assert b"even" in lib.wc_last_error()
    assert lib.wc_create_lattice(None, None, None) == -1
    # the largest accepted lattice has V/2 = 2^30 sites per parity; one more
    # doubling is refused before anything is allocated
    h = ctypes.c_void_p()
    rc = lib.wc_create_lattice((ctypes.c_int * 4)(2048, 2048, 1024, 2), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert b"too large" in lib.wc_last_error()


def test_null_handles_rejected(lib):
    lib.wc_load_links.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.wc_build_clover.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    lib.wc_solve.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_double] * 3 + [ctypes.c_void_p] * 2 + [ctypes.c_int,
                                                                                                   ctypes.c_void_p]
    assert lib.wc_load_links(None, None) == -1
    assert lib.wc_build_clover(None, 0.1, 1.0) == -1
    assert lib.wc_solve(None, None, 0.1, 1.0, 1e-10, None, None, 0, None) == -1
    lib.wc_spinor_bytes.restype = ctypes.c_size_t
    assert lib.wc_spinor_bytes(None, 1) == 0
    lib.wc_destroy_lattice(None)


def test_barrier_timeout_validated_on_host(lib):
    lib.wc_set_barrier_timeout.argtypes = [ctypes.c_double]
    assert lib.wc_set_barrier_timeout(-1.0) == -1
    assert lib.wc_set_barrier_timeout(float("nan")) == -1
    assert lib.wc_set_barrier_timeout(float("inf")) == -1
    assert lib.wc_set_barrier_timeout(2.0) == 0


def test_default_params(lib):
    import paper_1709_08785_amd as wc
    p = wc.SolveParams()
    lib.wc_solve_params_default(ctypes.byref(p))
    assert p.inner_prec == wc.FP32 and p.inner_maxit > 0 and p.outer_maxit > 0 and p.check_every > 0
    assert p.fixed_work == 0


def test_params_and_info_layout_match_header(tmp_path):
    # the binding's ctypes mirrors must agree with the C structs field by field
    import subprocess

    import paper_1709_08785_amd as wc
    here = os.path.dirname(os.path.abspath(__file__))
    inc = os.path.join(os.path.dirname(here), "include")
    fields = {"wc_solve_params": wc.SolveParams, "wc_solve_info": wc.SolveInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "wc.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {" ".join(l.split()[:-1]): int(l.split()[-1]) for l in out if l.strip()}
    for cname, cls in fields.items():
        assert got[cname + " size"] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got["%s %s" % (cname, f)] == getattr(cls, f).offset, (cname, f)
    p = wc.Lattice.default_params(outer="dc")
    assert p.outer == 1
    with pytest.raises(TypeError):
        wc.Lattice.default_params(not_a_parameter=1)


def test_binding_methods_are_callable_on_a_lattice():
    # the binding's Lattice methods take the arguments their docstrings name;
    # properties are reserved for read-only state
    import inspect

    import paper_1709_08785_amd as wc
    for name in ("set_block_size", "block_size", "tune_block_size", "set_link_recon", "solve", "solve_batch"):
        f = inspect.getattr_static(wc.Lattice, name)
        assert inspect.isfunction(f), name
    assert list(inspect.signature(wc.Lattice.set_block_size).parameters) == ["self", "threads"]
    assert isinstance(inspect.getattr_static(wc.Lattice, "link_recon"), property)
