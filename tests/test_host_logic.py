"""The library's shared index arithmetic, compiled for the host from its own
header and checked on the CPU: the XCD block remap is one-to-one for any
launch size, blocks_of covers every site, and the tiled even-odd addressing
covers each padded slab exactly once for the spinor (FP64, FP32, FP16 with
its scale plane) and full-link plane lists."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and not shutil.which("hipcc"), reason="hipcc not available")
def test_index_arithmetic_on_the_host(tmp_path):
    exe = tmp_path / "host_logic"
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1709_08785_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "host_logic.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
