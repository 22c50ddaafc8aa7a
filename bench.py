"""Benchmark: nested mixed-precision BiCGStab solve of the even-odd clover Wilson
system on one MI355X.

One step = one complete solve D x = b to true relative residual 1e-10 on the
32^3 x 64 lattice (links exp(0.3 i H), kappa = 0.135, c_SW = 1.0, one Gaussian
source): FP64 outer flexible BiCGStab around an FP32 inner BiCGStab (inner
tolerance 1e-6), links, clover and b resident in HBM when the clock starts.

Printed (one JSON line): the solve-wide effective bandwidth (algorithmic bytes
of every operator and BLAS kernel in the solve / solve time), the roofline of
the dominant kernel measured with HIP events on the library's stream, the
time to solution of the all-FP64 BiCGStab on the same system, and the FP64
oracle timed on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s (% HBM peak); time-to-1e-10 solve, mixed vs FP64 on 1 GPU"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C/C++/HIP source without its comments, runs of whitespace made one space;
    string and character literals are kept as they are."""
    out, i, n = [], 0, len(src)
    while i < n:
        ch = src[i]
        if ch in "\"'":
            j = i + 1
            while j < n and src[j] != ch:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def source_hash() -> str:
    """Hash of the kernel sources' code (comments and layout left out), which keys
    the stored HBM counters: they stay valid while the compiled code is the same."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1709_08785_amd", "csrc", "*"))):
        with open(f, encoding="utf-8") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + code_text(fh.read()).encode() + b"\0")
    return h.hexdigest()[:16]


def traffic_for(kernel: str, dims, recon: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/traffic.json), if one was taken on the current kernel
    sources for this lattice and FP32 link form; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    h = source_hash()
    for e in d.get("entries", []):
        if (e.get("source_hash") == h and e.get("kernel") == kernel and list(e.get("lattice", [])) == list(dims)
                and int(e.get("link_recon", 12)) == int(recon)):
            return e.get("hbm_bytes_per_launch")
    return None


# the paper's Table 1 flop counts per even site: MULT 2232 and D-hat 4512, so
# the second half of D-hat (MULT plus the xpay) 2280; axpy 96, dot 96, norm 48.
# One BiCGStab iteration (Algorithms 1 and 2 alike): two D-hat, three dots,
# three norms and six axpy-like updates.
T1_MULT, T1_DHAT = 2232, 4512
T1_ITER = 2 * T1_DHAT + 3 * 96 + 3 * 48 + 6 * 96


def table1_gflops(kname, Vh, avg_us):
    """GFLOPS of one stencil launch at the Table 1 count, or None for other kernels."""
    if kname.startswith("mult_hopinv"):
        f = T1_MULT
    elif kname.startswith("mult_dhat"):
        f = T1_DHAT - T1_MULT
    else:
        return None
    return round(f * Vh / (avg_us * 1e-6) / 1e9, 1)


def cpu_baseline(U, b, dims, kappa, csw, budget_s=20.0):
    """The FP64 oracle (plain C, OpenMP) applying the full D on the same lattice."""
    import numpy as np
    import oracle

    nthreads = oracle.num_threads()
    t0 = time.perf_counter()
    F = oracle.clover_field(U, dims, kappa, csw)
    t_clover = time.perf_counter() - t0
    n_apply = 0
    t0 = time.perf_counter()
    out = None
    while True:
        out = oracle.apply_D(U, F, kappa, b)
        n_apply += 1
        el = time.perf_counter() - t0
        if el > budget_s or n_apply >= 200:
            break
    el = time.perf_counter() - t0
    V = int(np.prod(dims))
    # algorithmic bytes of one full-lattice D in FP64: spinor in + out (2 x 192 B),
    # each of the 4V links once (4 x 144 B per site), one 2x36-real clover (576 B)
    bytes_per_site = 2 * 192 + 4 * 144 + 576
    gbs = n_apply * V * bytes_per_site / el / 1e9
    del F, out
    return {
        "value": round(gbs, 3),
        "unit": "GB/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": ("%d applications of the full FP64 operator D (oracle, precomputed clover; clover build "
                   "%.1f s not counted) on the %s lattice, %d B/site algorithmic" %
                   (n_apply, t_clover, "x".join(map(str, dims)), bytes_per_site)),
        "seconds": round(el, 3),
    }


def small_config():
    """The 8^4, kappa 0.12, c_SW 1.0 system (links seed 1001, Gaussian source seed
    2001) solved to 1e-10 by the GPU (FP32 inner, Algorithm 1 outer) and by the
    FP64 oracle's plain BiCGStab on the full D, on the host cores: context for
    the oracle's cost at the size its parity tests use."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_08785_amd as wc
    import synth

    dims, kappa, csw = (8, 8, 8, 8), 0.12, 1.0
    U = synth.random_links(dims, 0.3, 1001)
    b = synth.gaussian_source(dims, 2001)
    lat = wc.Lattice(dims)
    lat.load_links(torch.from_numpy(U).cuda())
    bd = torch.from_numpy(b).cuda()
    lat.solve(bd, kappa, csw, 1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = lat.solve(bd, kappa, csw, 1e-10)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    t0 = time.perf_counter()
    F = oracle.clover_field(U, dims, kappa, csw)
    x_ref, its, _ = oracle.solve(U, F, kappa, b, tol=1e-10)
    t_cpu = time.perf_counter() - t0
    xh = x.cpu().numpy()
    lat.close()
    return {"lattice": list(dims), "kappa": kappa, "tol": 1e-10, "gpu_s": round(t_gpu, 5),
            "gpu_inner_iters": info["inner_iters_total"], "oracle_s": round(t_cpu, 3), "oracle_iters": its,
            "oracle_threads": oracle.num_threads(),
            "solution_rel_diff": float(np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref))}


def collect(lat, res, suffix, fields=1):
    """Event-timed kernel statistics of lat into res (keys kernel + suffix); resets them."""
    st = lat.kernel_stats()
    for kname, v in st.items():
        if v["launches"]:
            avg_us = v["ms"] / v["launches"] * 1e3
            g = table1_gflops(kname, lat.volume // 2, avg_us)
            res[kname + suffix] = {
                "launches": v["launches"], "avg_us": round(avg_us, 2),
                "algorithmic_GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1),
                "frac_hbm": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "GFLOPS_table1": None if g is None else round(g * fields, 1),
                "bytes_per_launch": v["bytes"] / v["launches"]}
    lat.reset_kernel_stats()


def dslash_mode(args, dims):
    """Operator micro-benchmark: MULT and D-hat_ee in each precision, K launches each,
    timed with HIP events on the library stream; plus a device copy of known size
    (the calibration kernel for the HBM byte counters) and a stream with the
    stencil's 8:1 read/write mix, against which each operator's rate is also
    given as a fraction."""
    import numpy as np
    import torch

    import paper_1709_08785_amd as wc
    import synth

    dev = torch.device("cuda:0")
    # the links' exponential evaluated on the GPU (same draws as the host form)
    Ud = synth.random_links_torch(dims, 0.3, args.seed, device=dev)
    psi = synth.gaussian_source(dims, args.seed + 1000)
    lat = wc.Lattice(dims, device=dev)
    lat.load_links(Ud)
    del Ud
    lat.build_clover(args.kappa, args.csw)
    psid = torch.from_numpy(psi).to(dev)
    res = {}
    default_chunk = -1  # the lattice's own (tuned, else the default) chunk
    sweep = [int(v) for v in args.sweep_chunks.split(",")] if args.sweep_chunks else []
    wave_caps = [int(v) for v in args.sweep_wave_caps.split(",")] if args.sweep_wave_caps else []
    for name, prec, recon in [("fp32", wc.FP32, 12), ("fp16", wc.FP16, 12), ("fp64", wc.FP64, 12),
                              ("fp32", wc.FP32, 8), ("fp32", wc.FP32, 18)]:
        lat.set_link_recon(recon)
        eo = lat.pack(psid, prec)
        out = lat.new_eo(prec, 1)
        e_in = lat.parity_view(eo, 0, prec)
        o_in = lat.parity_view(eo, 1, prec)
        for chunk in [default_chunk] + [c for c in sweep if c != default_chunk]:
            lat.set_xcd_chunk(chunk)
            for w in range(3):
                lat.apply_mult(out, o_in, 0, prec)
                lat.apply_Dee_oo(out, e_in, prec)
            torch.cuda.synchronize()
            lat.reset_kernel_stats()
            lat.set_timing(True)
            for k in range(args.steps):
                lat.apply_mult(out, o_in, 0, prec)
            for k in range(args.steps):
                lat.apply_Dee_oo(out, e_in, prec)
            lat.set_timing(False)
            collect(lat, res, ("" if recon == 12 else "_recon%d" % recon) +
                    ("" if chunk == default_chunk else "_chunk%d" % chunk))
        lat.set_xcd_chunk(default_chunk)
        # the waves-per-CU cap: the FP64 stencil against no cap (it runs at 8 by
        # default), other caps on request
        caps = [0] if (prec == wc.FP64 and recon == 12) else []
        caps += [c for c in wave_caps if c not in caps]
        for cap in caps:
            lat.set_wave_cap(prec, cap)
            for w in range(3):
                lat.apply_mult(out, o_in, 0, prec)
                lat.apply_Dee_oo(out, e_in, prec)
            torch.cuda.synchronize()
            lat.reset_kernel_stats()
            lat.set_timing(True)
            for k in range(args.steps):
                lat.apply_mult(out, o_in, 0, prec)
            for k in range(args.steps):
                lat.apply_Dee_oo(out, e_in, prec)
            lat.set_timing(False)
            collect(lat, res, ("" if recon == 12 else "_recon%d" % recon) + "_cap%d" % cap)
        lat.set_wave_cap(prec, -1)
        del eo, out
    # the multi-system stencil: the 12 fields of the point-source batch on one
    # lattice, with 4 or 2 fields per thread and with one field per thread (the
    # fields' workgroups interleaved); algorithmic bytes per launch count the
    # links and clover once and every field's spinors (24S + 8L + C per site
    # for the MULT)
    nb = 12
    lat.set_link_recon(12)
    chunks = [default_chunk] + [c for c in sweep if c != default_chunk]
    for name, prec in (("fp32", wc.FP32), ("fp16", wc.FP16)):
        ins = [lat.pack(psid * (1.0 + 0.1 * k), prec) for k in range(nb)]
        outs = [lat.new_eo(prec, 1) for k in range(nb)]
        o_in = [lat.parity_view(e, 1, prec) for e in ins]
        e_in = [lat.parity_view(e, 0, prec) for e in ins]
        for chunk in chunks:
            lat.set_xcd_chunk(chunk)
            tag = "" if chunk == default_chunk else "_chunk%d" % chunk
            for gsz in (4, 2, 0):
                lat.set_multi_rhs(gsz)
                for w in range(2):
                    lat.apply_mult_batch(outs, o_in, 0, prec)
                    lat.apply_Dee_oo_batch(outs, e_in, prec)
                torch.cuda.synchronize()
                lat.reset_kernel_stats()
                lat.set_timing(True)
                for k in range(args.steps):
                    lat.apply_mult_batch(outs, o_in, 0, prec)
                for k in range(args.steps):
                    lat.apply_Dee_oo_batch(outs, e_in, prec)
                lat.set_timing(False)
                collect(lat, res, "_x%d_g%d%s" % (nb, gsz, tag), fields=nb)
        if sweep:
            # the 12 fields as sub-batches of 4 and 6 (the operator read once per
            # sub-batch), two and four fields per thread
            lat.set_xcd_chunk(default_chunk)
            for sub in (4, 6):
                for gsz in (4, 2):
                    lat.set_multi_rhs(gsz)
                    for w in range(2):
                        lat.apply_mult_batch(outs[:sub], o_in[:sub], 0, prec)
                    torch.cuda.synchronize()
                    lat.reset_kernel_stats()
                    lat.set_timing(True)
                    for k in range(args.steps):
                        for j in range(0, nb, sub):
                            lat.apply_mult_batch(outs[j:j + sub], o_in[j:j + sub], 0, prec)
                    lat.set_timing(False)
                    collect(lat, res, "_x%d_in%d_g%d" % (nb, sub, gsz), fields=sub)
        del ins, outs, o_in, e_in
    lat.set_xcd_chunk(default_chunk)
    lat.set_multi_rhs(-1)
    # calibration copy: 1 GiB read + 1 GiB written
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for k in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.steps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    copy_gbs = 2 * 4 * n / (ms * 1e-3) / 1e9
    res["copy_1GiB"] = {"avg_us": round(ms * 1e3, 2), "GBs": round(copy_gbs, 1),
                        "bytes_read": 4 * n, "bytes_written": 4 * n}
    # torch's column sum as a stream with the stencil's read/write mix (8 reads
    # per write: the MULT reads 768 B and writes 96 B per site in FP32): 1 GiB
    # summed in 8 rows
    col = torch.empty(n // 8, dtype=torch.float32, device=dev)
    a8 = a.view(8, n // 8)
    for k in range(3):
        torch.sum(a8, dim=0, out=col)
    torch.cuda.synchronize()
    e0.record()
    for k in range(args.steps):
        torch.sum(a8, dim=0, out=col)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    mix_gbs = (4 * n + 4 * n // 8) / (ms * 1e-3) / 1e9
    res["read8_write1_1GiB"] = {"avg_us": round(ms * 1e3, 2), "GBs": round(mix_gbs, 1), "bytes_read": 4 * n,
                                "bytes_written": 4 * n // 8}
    # each operator's rate also as a fraction of the two measured torch streams
    for k, v in res.items():
        if "algorithmic_GBs" in v:
            v["frac_copy"] = round(v["algorithmic_GBs"] / copy_gbs, 4)
            v["frac_read8_write1_stream"] = round(v["algorithmic_GBs"] / mix_gbs, 4)
    print(json.dumps({"mode": "dslash", "lattice": list(dims), "kernels": res}), flush=True)


def batch_mode(args):
    """Batched solves: (a) 12 spin-colour point sources on one 32^3x64 lattice,
    (b) one Gaussian source on each of 16^4, 24^3x48 and 32^3x64.  Each set is
    solved together (one launch per phase, chunk graphs) and, for comparison,
    one system after another; FP32 inner / FP64 outer to true residual tol,
    and the point sources also with the FP16-storage inner solve."""
    import torch

    import paper_1709_08785_amd as wc
    import synth

    dev = torch.device("cuda:0")
    out = {"mode": "batch", "tol": args.tol, "inner": "fp32", "kappa": 0.135, "csw": 1.0}
    kappa, csw = 0.135, 1.0

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # (a) 12 point sources on 32^3 x 64
    dims = (32, 32, 32, 64)
    lat = wc.Lattice(dims, device=dev)
    lat.load_links(torch.from_numpy(synth.random_links(dims, 0.3, 1004)).to(dev))
    lat.build_clover(kappa, csw)
    bs = [torch.from_numpy(synth.point_source(dims, al, a)).to(dev) for al in range(4) for a in range(3)]
    # the batch with the multi-system stencil at 2 fields per thread, and with
    # one field per thread (interleaved workgroups), before the default 4
    by_g = {}
    for gsz in (0, 4, 2):
        lat.set_multi_rhs(gsz)
        lat.solve_batch(bs, kappa, csw, args.tol)  # warm-up (allocation, graph recording)
        (xs, infos), t_batch = timed(lambda: lat.solve_batch(bs, kappa, csw, args.tol))
        by_g[gsz] = {"batched_s": round(t_batch, 4), "max_true_rel_residual": max(i["true_rel_residual"] for i in infos),
                     "inner_iters": [i["inner_iters_total"] for i in infos]}
        log("point sources, %d fields per thread: %s" % (gsz, json.dumps(by_g[gsz])))
    lat.set_multi_rhs(-1)  # the precision's default (2 in FP32): the last timing above
    lat.solve(bs[0], kappa, csw, args.tol)
    singles, t_seq = timed(lambda: [lat.solve(b, kappa, csw, args.tol) for b in bs])
    # per-kernel accounting of one batched solve (eager, HIP events)
    lat.reset_kernel_stats()
    lat.set_timing(True)
    lat.solve_batch(bs, kappa, csw, args.tol)
    lat.set_timing(False)
    st = lat.kernel_stats()
    tot_bytes = sum(v["bytes"] for v in st.values())
    tot_ms = sum(v["ms"] for v in st.values())
    out["point_sources_32x32x32x64"] = {
        "systems": len(bs), "batched_s": round(t_batch, 4), "sequential_s": round(t_seq, 4),
        "speedup": round(t_seq / t_batch, 3), "s_per_system_batched": round(t_batch / len(bs), 4),
        "fields_per_thread": lat.multi_rhs(wc.FP32), "by_fields_per_thread": {str(k): v for k, v in by_g.items()},
        "max_true_rel_residual": max(i["true_rel_residual"] for i in infos),
        "inner_iters": [i["inner_iters_total"] for i in infos],
        "algorithmic_GBs_batched_kernels": round(tot_bytes / (tot_ms * 1e-3) / 1e9, 1),
        "kernels": {k: {"launches": v["launches"], "avg_us": round(v["ms"] / v["launches"] * 1e3, 2),
                        "GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)}
                    for k, v in st.items() if v["launches"]},
    }
    log("point sources:", json.dumps(out["point_sources_32x32x32x64"]))
    # the same 12 sources with the FP16-storage inner solve (4 fields per thread),
    # batched and one after another
    lat.solve_batch(bs, kappa, csw, args.tol, inner_prec=wc.FP16)
    (xs16, inf16), t_b16 = timed(lambda: lat.solve_batch(bs, kappa, csw, args.tol, inner_prec=wc.FP16))
    lat.solve(bs[0], kappa, csw, args.tol, inner_prec=wc.FP16)
    _, t_s16 = timed(lambda: [lat.solve(b, kappa, csw, args.tol, inner_prec=wc.FP16) for b in bs])
    out["point_sources_32x32x32x64_fp16_inner"] = {
        "batched_s": round(t_b16, 4), "sequential_s": round(t_s16, 4), "speedup": round(t_s16 / t_b16, 3),
        "fields_per_thread": lat.multi_rhs(wc.FP16), "vs_fp32_batched": round(t_batch / t_b16, 3),
        "max_true_rel_residual": max(i["true_rel_residual"] for i in inf16),
        "inner_iters": [i["inner_iters_total"] for i in inf16],
    }
    log("point sources, FP16 inner:", json.dumps(out["point_sources_32x32x32x64_fp16_inner"]))
    del xs, xs16, singles, bs
    lat.close()
    torch.cuda.empty_cache()

    # (b) uneven lattices, one Gaussian source each
    lats, bs = [], []
    for i, d in enumerate([(16, 16, 16, 16), (24, 24, 24, 48), (32, 32, 32, 64)]):
        l = wc.Lattice(d, device=dev)
        l.load_links(torch.from_numpy(synth.random_links(d, 0.3, 1004 + 10 * i)).to(dev))
        l.build_clover(kappa, csw)
        lats.append(l)
        bs.append(torch.from_numpy(synth.gaussian_source(d, 2004 + 10 * i)).to(dev))
    wc.solve_multi(lats, bs, [kappa] * 3, [csw] * 3, args.tol)
    (xs, infos), t_batch = timed(lambda: wc.solve_multi(lats, bs, [kappa] * 3, [csw] * 3, args.tol))
    singles, t_seq = timed(lambda: [l.solve(b, kappa, csw, args.tol) for l, b in zip(lats, bs)])
    out["uneven_16^4_24^3x48_32^3x64"] = {
        "batched_s": round(t_batch, 4), "sequential_s": round(t_seq, 4), "speedup": round(t_seq / t_batch, 3),
        "max_true_rel_residual": max(i["true_rel_residual"] for i in infos),
        "inner_iters": [i["inner_iters_total"] for i in infos],
    }
    # small lattice alone: launch-bound, where the chunk graphs matter
    small, b0 = lats[0], bs[0]
    small.solve(b0, kappa, csw, args.tol, use_graph=1)
    (_, ig), t_graph = timed(lambda: small.solve(b0, kappa, csw, args.tol, use_graph=1))
    small.solve(b0, kappa, csw, args.tol, use_graph=0)
    (_, ie), t_eager = timed(lambda: small.solve(b0, kappa, csw, args.tol, use_graph=0))
    out["16^4_single_solve"] = {"graph_s": round(t_graph, 5), "eager_s": round(t_eager, 5),
                                "speedup_graph": round(t_eager / t_graph, 3), "inner_iters": ig["inner_iters_total"]}
    print(json.dumps(out), flush=True)


def inner_mode(args):
    """Algorithm 2 (launched loop with chunk graphs) against the pipelined inner
    BiCGStab (two reduction phases per iteration instead of four, more vector
    traffic) and against the one-launch loop (a cooperative kernel, where the
    lattice fits), from the launch-bound 8^4 to the bandwidth-bound 32^3x64:
    FP32 inner, Algorithm 1 outer, kappa 0.13, c_SW 1.0, Gaussian source, tol
    on the true residual."""
    import torch

    import paper_1709_08785_amd as wc
    import synth

    dev = torch.device("cuda:0")
    kappa, csw = 0.13, 1.0
    rows = {}
    for i, d in enumerate([(8, 8, 8, 8), (16, 16, 16, 16), (24, 24, 24, 48), (32, 32, 32, 64)]):
        lat = wc.Lattice(d, device=dev)
        lat.load_links(torch.from_numpy(synth.random_links(d, 0.3, 1100 + i)).to(dev))
        lat.build_clover(kappa, csw)
        b = torch.from_numpy(synth.gaussian_source(d, 2100 + i)).to(dev)
        row = {}
        for name in ("bicgstab", "pipelined", "persistent"):
            kw = {"persistent": 1} if name == "persistent" else {"inner_method": name}
            lat.solve(b, kappa, csw, args.tol, **kw)
            reps = 20 if d[0] <= 16 else 3
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(reps):
                x, info = lat.solve(b, kappa, csw, args.tol, **kw)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / reps
            row[name] = {"ms": round(el * 1e3, 3), "inner_iters": info["inner_iters_total"],
                         "inner_calls": info["inner_calls"], "outer_iters": info["outer_iters"],
                         "us_per_inner_iter": round(el * 1e6 / info["inner_iters_total"], 2),
                         "true_rel_residual": info["true_rel_residual"],
                         "one_launch_inner_calls": info["persistent_calls"]}
            log("inner %s %s %s" % ("x".join(map(str, d)), name, json.dumps(row[name])))
        row["pipelined_speedup"] = round(row["bicgstab"]["ms"] / row["pipelined"]["ms"], 3)
        row["persistent_speedup"] = round(row["bicgstab"]["ms"] / row["persistent"]["ms"], 3)
        rows["x".join(map(str, d))] = row
        lat.close()
    print(json.dumps({"mode": "inner", "kappa": kappa, "csw": csw, "tol": args.tol, "inner": "fp32",
                      "lattices": rows}), flush=True)


def precisions_mode(args):
    """The three precision forms on the 48^3x96 lattice (kappa 0.1355, c_SW 1.0,
    Z2 source), all refined in FP64 to true relative residual tol: FP16-storage
    inner, FP32 inner, and the all-FP64 BiCGStab; then FP32 inner with
    reconstruct-8 links, and the defect-correction outer with FP16 and with
    reconstruct-8 FP32 inner solves.  Each solution's residual is also computed
    by the FP64 oracle on the host."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_08785_amd as wc
    import synth

    dims = (48, 48, 48, 96)
    kappa, csw = 0.1355, 1.0
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    Ud = synth.random_links_torch(dims, 0.3, 1003, device=dev)
    b = synth.z2_source(dims, 2003)
    log("48^3x96 inputs in %.1f s" % (time.perf_counter() - t0))
    lat = wc.Lattice(dims, device=dev)
    lat.load_links(Ud)
    lat.build_clover(kappa, csw)
    U = Ud.cpu().numpy()
    del Ud
    bd = torch.from_numpy(b).to(dev)
    # the three forms of the paper's method (flexible BiCGStab outer), then the
    # same with reconstruct-8 FP32 links and with the defect-correction outer
    forms = [("fp16", 12, dict(inner_prec=wc.FP16)), ("fp32", 12, dict(inner_prec=wc.FP32)),
             ("fp64", 12, dict(inner_prec=wc.FP64)), ("fp32_recon8", 8, dict(inner_prec=wc.FP32)),
             ("fp16_dc", 12, dict(inner_prec=wc.FP16, outer="dc")),
             ("fp32_recon8_dc", 8, dict(inner_prec=wc.FP32, outer="dc"))]
    res = {}
    xs = {}
    for name, recon, kw in forms:
        lat.set_link_recon(recon)
        lat.solve(bd, kappa, csw, args.tol, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = lat.solve(bd, kappa, csw, args.tol, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        xh = x.cpu().numpy()
        r, bn = oracle.residual(U, kappa, csw, b, xh)
        xs[name] = xh
        ip = kw["inner_prec"]
        res[name] = {"seconds": round(el, 4), "inner_iters": info["inner_iters_total"],
                     "outer_iters": info["outer_iters"], "restarts": info["restarts"],
                     "true_rel_residual_gpu": info["true_rel_residual"], "true_rel_residual_oracle": r / bn,
                     "threads_per_block": info["block_size"], "xcd_chunk_tiles": lat.xcd_chunk(ip),
                     "waves_per_cu_cap": {"mult": lat.wave_cap(ip), "dhat": lat.wave_cap(ip, dhat=True)}}
        log(name, json.dumps(res[name]))
        del x
    lat.set_link_recon(12)
    for name in [f[0] for f in forms if f[0] != "fp64"]:
        res[name]["solution_rel_diff_vs_fp64"] = float(np.linalg.norm(xs[name] - xs["fp64"]) /
                                                       np.linalg.norm(xs["fp64"]))
        res[name]["speedup_vs_fp64"] = round(res["fp64"]["seconds"] / res[name]["seconds"], 3)
    print(json.dumps({"mode": "precisions", "lattice": list(dims), "kappa": kappa, "csw": csw, "tol": args.tol,
                      "source": "Z2", "forms": res, "oracle_threads": oracle.num_threads()}), flush=True)


def tune_mode(args):
    """The launch-shape tuner on 8^4 .. 32^3x64: its microseconds per stencil pair
    (F^-1 H, then the D-hat half with its fused dot) at 64, 128 and 256 threads
    per block in each precision, its choice, and the nested solve (FP32 inner,
    Algorithm 1 outer, kappa 0.13, c_SW 1, Gaussian source, tol) at the tuned
    size against 256 pinned, and at 2 to 32 inner iterations between host
    convergence reads."""
    import torch

    import paper_1709_08785_amd as wc
    import synth

    kappa, csw = 0.13, 1.0
    out = {"mode": "tune", "kappa": kappa, "csw": csw, "tol": args.tol, "lattices": {}}
    for dims in [(8, 8, 8, 8), (16, 16, 16, 16), (24, 24, 24, 48), (32, 32, 32, 64)]:
        name = "x".join(map(str, dims))
        lat = wc.Lattice(dims)
        lat.load_links(torch.from_numpy(synth.random_links(dims, 0.3, 1070)).cuda())
        lat.build_clover(kappa, csw)
        row = {"tuner": {}}
        for pname, prec in (("fp32", wc.FP32), ("fp16", wc.FP16), ("fp64", wc.FP64)):
            r = lat.tune_block_size(prec)
            row["tuner"][pname] = {"us_per_pair": {str(k): round(v, 2) for k, v in r["us_per_pair"].items()},
                                   "threads": r["threads"], "xcd_chunk_tiles": r["chunk"],
                                   "waves_per_cu_cap": r["wave_cap"]}
        b = torch.from_numpy(synth.gaussian_source(dims, 2070)).cuda()
        reps = 20 if dims[0] <= 16 else 3
        for label, pin, chunk in (("pinned_256_chunk32", 256, 32), ("tuned", 0, -1)):
            lat.set_block_size(pin)
            lat.set_xcd_chunk(chunk)
            lat.solve(b, kappa, csw, args.tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(reps):
                x, info = lat.solve(b, kappa, csw, args.tol)
            torch.cuda.synchronize()
            row[label] = {"ms": round((time.perf_counter() - t0) / reps * 1e3, 3), "threads": info["block_size"],
                          "xcd_chunk_tiles": lat.xcd_chunk(wc.FP32),
                          "inner_iters": info["inner_iters_total"], "true_rel_residual": info["true_rel_residual"]}
        row["speedup_tuned"] = round(row["pinned_256_chunk32"]["ms"] / row["tuned"]["ms"], 3)
        # inner iterations queued between host convergence reads: fewer reads
        # against more launches queued after convergence (they return at once)
        row["check_every_ms"] = {}
        for ce in (2, 4, 8, 16, 32):
            lat.solve(b, kappa, csw, args.tol, check_every=ce)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(reps):
                x, info = lat.solve(b, kappa, csw, args.tol, check_every=ce)
            torch.cuda.synchronize()
            row["check_every_ms"][str(ce)] = round((time.perf_counter() - t0) / reps * 1e3, 3)
        log("tune %s %s" % (name, json.dumps(row)))
        out["lattices"][name] = row
        lat.close()
    print(json.dumps(out), flush=True)


def host_info():
    """Model name and core counts of the host CPU (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "usable_cpus": aff,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_mode(args):
    """The FP64 oracle on the host cores, as it stands (never tuned): one full D
    and one D-hat_ee at 8^4 and 32^3x64, with one thread and with all, then the
    full solves to 1e-10 of the 8^4 (kappa 0.12, links 1001, source 2001) and
    32^3x64 (kappa 0.135, links 1002, source 2002) systems with all threads,
    beside the GPU's solves of the same systems (FP32 inner / FP64 outer, and
    all-FP64).  Rates use the algorithmic bytes of the FP64 operator (full D:
    1536 B per site; D-hat_ee: 4416 B per even site) and the paper's Table 1
    flop counts (2232 per site for an operator application over all sites,
    4512 per even site for D-hat_ee)."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_08785_amd as wc
    import synth

    csw = 1.0
    nall = oracle.num_threads()
    out = {"mode": "oracle", "host": host_info(), "oracle_threads_all": nall, "apply": {}, "solve": {}}
    for dims, kappa, seed in [((8, 8, 8, 8), 0.12, 1001), ((32, 32, 32, 64), 0.135, 1002)]:
        name = "x".join(map(str, dims))
        V = int(np.prod(dims))
        U = synth.random_links(dims, 0.3, seed)
        b = synth.gaussian_source(dims, seed + 1000)
        F = oracle.clover_field(U, dims, kappa, csw)
        Finv = oracle.site_invert(F)
        be = oracle.restrict(b, 0)
        row = {}
        for nt in sorted({1, nall}):
            oracle.set_num_threads(nt)
            reps = 20 if V < 100000 else 1
            t0 = time.perf_counter()
            for r in range(reps):
                oracle.apply_D(U, F, kappa, b)
            t_d = (time.perf_counter() - t0) / reps
            t0 = time.perf_counter()
            for r in range(reps):
                oracle.dhat_ee(U, Finv, kappa, be)
            t_h = (time.perf_counter() - t0) / reps
            row["threads_%d" % nt] = {
                "D_s": round(t_d, 5), "D_GBs": round(V * 1536 / t_d / 1e9, 3),
                "D_GFLOPS": round(V * 2232 / t_d / 1e9, 3),
                "dhat_s": round(t_h, 5), "dhat_GBs": round(V / 2 * 4416 / t_h / 1e9, 3),
                "dhat_GFLOPS": round(V / 2 * 4512 / t_h / 1e9, 3)}
            log("oracle %s threads %d: %s" % (name, nt, json.dumps(row["threads_%d" % nt])))
        oracle.set_num_threads(nall)
        out["apply"][name] = row
        # the full solves: oracle (all threads) and GPU
        t0 = time.perf_counter()
        x_ref, its, relres = oracle.solve(U, F, kappa, b, tol=args.tol)
        t_or = time.perf_counter() - t0
        log("oracle solve %s: %.1f s, %d iterations, true relres %.2e" % (name, t_or, its, relres))
        lat = wc.Lattice(dims)
        lat.load_links(torch.from_numpy(U).cuda())
        bd = torch.from_numpy(b).cuda()
        gpu = {}
        for form, kw in [("mixed_fp32_inner", {}), ("fp64", {"inner_prec": wc.FP64})]:
            lat.solve(bd, kappa, csw, args.tol, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = lat.solve(bd, kappa, csw, args.tol, **kw)
            torch.cuda.synchronize()
            t_g = time.perf_counter() - t0
            xh = x.cpu().numpy()
            gpu[form] = {"seconds": round(t_g, 5), "inner_iters": info["inner_iters_total"],
                         "true_rel_residual": info["true_rel_residual"],
                         "solution_rel_diff_vs_oracle": float(np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)),
                         "oracle_over_gpu": round(t_or / t_g, 1)}
        lat.close()
        out["solve"][name] = {"kappa": kappa, "tol": args.tol, "oracle_s": round(t_or, 3), "oracle_iters": its,
                              "oracle_true_rel_residual": relres, "oracle_threads": nall, "gpu": gpu}
        del U, b, F, Finv, be, x_ref
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["solve", "dslash", "batch", "precisions", "inner", "oracle", "tune"],
                    default="solve")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=str, default="32,32,32,64")
    ap.add_argument("--kappa", type=float, default=0.135)
    ap.add_argument("--csw", type=float, default=1.0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner-tol", type=float, default=1e-6)
    ap.add_argument("--inner", type=str, default="fp32")
    ap.add_argument("--recon", type=int, default=12, choices=[12, 8, 18])
    ap.add_argument("--no-fp64-arm", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1002)
    ap.add_argument("--sweep-chunks", type=str, default="",
                    help="dslash mode: also time the stencils at these XCD chunks (tiles, comma-separated; "
                         "0 = one slab per XCD) and the batched ones at sub-batch sizes")
    ap.add_argument("--wave-cap", type=int, default=None,
                    help="waves-per-CU cap of the inner precision's one-system stencils in the timed solve "
                         "(0 = none; default: the library's)")
    ap.add_argument("--sweep-wave-caps", type=str, default="",
                    help="dslash mode: also time the one-system stencils of every precision at these "
                         "waves-per-CU caps (comma-separated; 0 = no cap)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(it runs one process's share of a lattice on one GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_08785_amd as wc
    import synth

    dims = tuple(int(v) for v in args.dims.split(","))
    if args.mode == "dslash":
        dslash_mode(args, dims)
        return
    if args.mode == "batch":
        batch_mode(args)
        return
    if args.mode == "precisions":
        precisions_mode(args)
        return
    if args.mode == "inner":
        inner_mode(args)
        return
    if args.mode == "oracle":
        oracle_mode(args)
        return
    if args.mode == "tune":
        tune_mode(args)
        return
    t0 = time.perf_counter()
    U = synth.random_links(dims, 0.3, args.seed)
    b = synth.gaussian_source(dims, args.seed + 1000)
    log("inputs generated in %.1f s" % (time.perf_counter() - t0))

    dev = torch.device("cuda:0")
    lat = wc.Lattice(dims, device=dev)
    Ud = torch.from_numpy(U).to(dev)
    bd = torch.from_numpy(b).to(dev)
    lat.load_links(Ud)
    lat.build_clover(args.kappa, args.csw)
    lat.set_link_recon(args.recon)
    del Ud
    torch.cuda.synchronize()
    inner = wc._prec(args.inner)
    if args.wave_cap is not None:
        lat.set_wave_cap(inner, args.wave_cap)
    solve_kw = dict(inner_prec=inner, inner_tol=args.inner_tol)

    for w in range(args.warmup):
        x, info = lat.solve(bd, args.kappa, args.csw, args.tol, **solve_kw)
        log("warmup %d: %s" % (w, json.dumps(info)))

    # the timed steps: plain solves (inner-loop chunks replayed as graphs, no events)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        x, info = lat.solve(bd, args.kappa, args.csw, args.tol, **solve_kw)
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s, info in enumerate(infos):
        log("step %d: %s" % (s, json.dumps(info)))
    ms_per_step = wall / args.steps * 1e3
    # one more solve of the same system with every launch between HIP events:
    # per-kernel times and the algorithmic bytes of the work actually done
    # (launches queued after convergence return at once and are not counted).
    # The solve is deterministic, so it repeats the timed steps' iterations.
    lat.reset_kernel_stats()
    lat.set_timing(True)
    _, info_t = lat.solve(bd, args.kappa, args.csw, args.tol, **solve_kw)
    lat.set_timing(False)
    stats = lat.kernel_stats()
    assert info_t["inner_iters_total"] == infos[-1]["inner_iters_total"], (info_t, infos[-1])
    bytes_per_solve = sum(v["bytes"] for v in stats.values())
    value = bytes_per_solve * args.steps / wall / 1e9

    # dominant kernel by total event time
    dom_name, dom = max(((k, v) for k, v in stats.items() if v["launches"] > 0), key=lambda kv: kv[1]["ms"])
    per_launch_bytes = dom["bytes"] / dom["launches"]
    avg_ms = dom["ms"] / dom["launches"]
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    hbm = traffic_for(dom_name, dims, args.recon)
    roofline = {
        "bound": "hbm",
        "kernel": dom_name,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": hbm,
        "avg_launch_us": round(avg_ms * 1e3, 2),
        "algorithmic_bytes_per_launch": per_launch_bytes,
    }
    kern = {k: {"launches": v["launches"], "avg_us": round(v["ms"] / v["launches"] * 1e3, 2),
                "GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1),
                "GFLOPS_table1": table1_gflops(k, lat.volume // 2, v["ms"] / v["launches"] * 1e3)}
            for k, v in stats.items() if v["launches"] > 0}
    # the whole step at the Table 1 counts: every inner and outer iteration
    # costs two D-hat and the BLAS-1 of one BiCGStab iteration per even site
    step_flops = T1_ITER * (lat.volume // 2) * (infos[-1]["inner_iters_total"] + infos[-1]["outer_iters"])

    # the all-FP64 arm on the same system
    fp64 = None
    fp16 = None
    recon8 = None
    dc = None
    if not args.no_fp64_arm:
        x64, info64 = lat.solve(bd, args.kappa, args.csw, args.tol, inner_prec=wc.FP64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x64, info64 = lat.solve(bd, args.kappa, args.csw, args.tol, inner_prec=wc.FP64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        log("fp64 arm: %s" % json.dumps(info64))
        diff = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        fp64 = {"seconds": round(t64, 4), "iterations": info64["inner_iters_total"],
                "true_rel_residual": info64["true_rel_residual"], "mixed_vs_fp64_solution_rel_diff": diff}
        # the FP16-storage inner form on the same system (reported beside the FP32 step)
        lat.solve(bd, args.kappa, args.csw, args.tol, inner_prec=wc.FP16)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x16, info16 = lat.solve(bd, args.kappa, args.csw, args.tol, inner_prec=wc.FP16)
        torch.cuda.synchronize()
        t16 = time.perf_counter() - t1
        log("fp16 arm: %s" % json.dumps(info16))
        fp16 = {"seconds": round(t16, 4), "inner_iters": info16["inner_iters_total"],
                "outer_iters": info16["outer_iters"], "true_rel_residual": info16["true_rel_residual"],
                "solution_rel_diff_vs_fp64": float(torch.linalg.norm(x16 - x64) / torch.linalg.norm(x64)),
                "speedup_vs_fp64": round(t64 / t16, 3)}
        del x16
        # further forms of the same solve: reconstruct-8 links in the FP32 inner
        # stencil, and the defect-correction outer iteration
        if args.recon == 12:
            def arm(prec, recon, outer):
                lat.set_link_recon(recon)
                lat.solve(bd, args.kappa, args.csw, args.tol, inner_prec=prec, outer=outer)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                xa, ia = lat.solve(bd, args.kappa, args.csw, args.tol, inner_prec=prec, outer=outer)
                torch.cuda.synchronize()
                ta = time.perf_counter() - t1
                lat.set_link_recon(args.recon)
                log("arm %s recon %d %s: %s" % (prec, recon, outer, json.dumps(ia)))
                return {"seconds": round(ta, 4), "inner_iters": ia["inner_iters_total"],
                        "inner_calls": ia["inner_calls"], "outer_iters": ia["outer_iters"],
                        "true_rel_residual": ia["true_rel_residual"],
                        "solution_rel_diff_vs_fp64": float(torch.linalg.norm(xa - x64) / torch.linalg.norm(x64)),
                        "speedup_vs_fp64": round(t64 / ta, 3)}
            recon8 = {"fp32_inner": arm(wc.FP32, 8, "bicgstab")}
            dc = {"fp32_inner": arm(wc.FP32, 12, "dc"), "fp32_inner_recon8": arm(wc.FP32, 8, "dc"),
                  "fp16_inner": arm(wc.FP16, 12, "dc")}

    cpu = None
    small = None
    if not args.no_cpu_baseline:
        del x
        torch.cuda.synchronize()
        cpu = cpu_baseline(U, b, dims, args.kappa, args.csw)
        small = small_config()

    last = infos[-1]
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if inner == wc.FP32 else ("f16s+f32+f64" if inner == wc.FP16 else "f64"),
        "data": "synthetic",
        "config": {"workload": "nested BiCGStab solve, %s lattice, exp(0.3 i H) links, kappa %g, c_SW %g, "
                               "Gaussian source, %s inner (tol %g) / FP64 outer, true residual %g"
                               % ("x".join(map(str, dims)), args.kappa, args.csw, args.inner.upper(),
                                  args.inner_tol, args.tol),
                   "lattice": list(dims), "kappa": args.kappa, "csw": args.csw, "tol": args.tol,
                   "inner": args.inner, "inner_tol": args.inner_tol, "link_recon": args.recon,
                   "threads_per_block": infos[-1]["block_size"], "xcd_chunk_tiles": lat.xcd_chunk(inner),
                   "waves_per_cu_cap": {"mult": lat.wave_cap(inner), "dhat": lat.wave_cap(inner, dhat=True)}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "small_config_8x8x8x8": small,
        "time_to_solution_s": {"mixed": round(ms_per_step / 1e3, 4), "fp64": fp64["seconds"] if fp64 else None,
                               "mixed_fp16_inner": fp16["seconds"] if fp16 else None,
                               "mixed_recon8": recon8["fp32_inner"]["seconds"] if recon8 else None,
                               "dc_fp32_inner": dc["fp32_inner"]["seconds"] if dc else None,
                               "dc_fp32_inner_recon8": dc["fp32_inner_recon8"]["seconds"] if dc else None,
                               "dc_fp16_inner": dc["fp16_inner"]["seconds"] if dc else None},
        "speedup_mixed_vs_fp64": round(fp64["seconds"] / (ms_per_step / 1e3), 3) if fp64 else None,
        "solve_GFLOPS_table1": round(step_flops / (ms_per_step * 1e-3) / 1e9, 1),
        "fp64_arm": fp64,
        "fp16_inner_arm": fp16,
        "recon8_arms": recon8,
        "defect_correction_arms": dc,
        "solve": {"outer_iters": last["outer_iters"], "inner_iters": last["inner_iters_total"],
                  "inner_calls": last["inner_calls"], "restarts": last["restarts"],
                  "true_rel_residual": last["true_rel_residual"], "dslash_count": last["dslash_count"]},
        "kernels": kern,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
