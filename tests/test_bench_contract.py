"""Host-side parts of the benchmark contract: more than one GPU is refused
with a message before anything touches a device, and the Table 1 flop
bookkeeping and roofline helpers give the paper's counts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_table1_counts():
    # Table 1: MULT 2232 and D-hat 4512 flops per site; axpy 96, dot 96, norm 48
    assert bench.T1_MULT == 2232 and bench.T1_DHAT == 4512
    assert bench.T1_ITER == 2 * 4512 + 3 * 96 + 3 * 48 + 6 * 96 == 10032
    # 1M sites at 1 ms: 2.232 TFLOPS for a MULT, 2.28 for the D-hat half
    assert bench.table1_gflops("mult_hopinv_fp32", 10 ** 6, 1000.0) == 2232.0
    assert bench.table1_gflops("mult_dhat_fp16", 10 ** 6, 1000.0) == 2280.0
    assert bench.table1_gflops("blas", 10 ** 6, 1000.0) is None


def test_traffic_is_null_for_other_sources_or_shapes(tmp_path, monkeypatch):
    # HBM bytes from the stored counters are used only while the kernel
    # sources hash to the value they were taken on, and only for the lattice
    # and link form they were taken on
    import json
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"source_hash": "abcdabcdabcdabcd", "lattice": [32, 32, 32, 64], "link_recon": 12,
             "kernel": "mult_dhat_fp32", "hbm_bytes_per_launch": 123}
    (prof / "traffic.json").write_text(json.dumps({"entries": [entry]}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "abcdabcdabcdabcd")
    assert bench.traffic_for("mult_dhat_fp32", (32, 32, 32, 64), 12) == 123
    assert bench.traffic_for("mult_dhat_fp32", (48, 48, 48, 96), 12) is None
    assert bench.traffic_for("mult_dhat_fp32", (32, 32, 32, 64), 8) is None
    assert bench.traffic_for("mult_hopinv_fp32", (32, 32, 32, 64), 12) is None
    monkeypatch.setattr(bench, "source_hash", lambda: "0000000000000000")
    assert bench.traffic_for("mult_dhat_fp32", (32, 32, 32, 64), 12) is None


def test_source_hash_follows_code_not_comments(tmp_path, monkeypatch):
    # the stored HBM counters are keyed by the kernel sources' code: editing a
    # comment keeps the key, editing code changes it
    assert bench.code_text('a // c\nb /* x\n y */ c "//s" \'/\' d') == 'a b c "//s" \'/\' d'
    src = os.path.join(bench.ROOT, "paper_1709_08785_amd", "csrc")
    dst = tmp_path / "paper_1709_08785_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in sorted(os.listdir(src)):
        if os.path.isfile(os.path.join(src, name)):
            (dst / name).write_text(open(os.path.join(src, name), encoding="utf-8").read(), encoding="utf-8")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    f = dst / "reduce.hpp"
    text = f.read_text(encoding="utf-8")
    f.write_text("// another comment\n" + text.replace("// ", "//  ") + "\n/* trailing */\n", encoding="utf-8")
    assert bench.source_hash() == h0
    f.write_text(text.replace("kBlock = 256", "kBlock = 128"), encoding="utf-8")
    assert bench.source_hash() != h0
