"""Python binding of the gfx950 Wilson-clover quark-solver library (libwc.so).

Argument marshalling only: every step of the operator and the solvers runs in
the library's HIP kernels.  torch supplies device memory and the stream.  The
binding refuses to work when the built library is missing; there is no CPU
path.

Fields are torch tensors on the GPU in the canonical layouts of ``include/wc.h``:
links ``complex128 (4, Lt, Lz, Ly, Lx, 3, 3)``, spinors
``complex128 (Lt, Lz, Ly, Lx, 4, 3)``.  Even-odd (EO) fields are opaque byte
tensors (``uint8``) in the library's structure-of-arrays layout.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import torch

__all__ = ["Lattice", "SolveParams", "FP64", "FP32", "FP16", "WCError", "library_path", "load_library", "solve",
           "solve_multi"]

FP64, FP32, FP16 = 0, 1, 2
_PREC_NAMES = {"fp64": FP64, "fp32": FP32, "fp16": FP16}
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libwc.so")
_lib = None

STATUS = {0: "WC_OK", -1: "WC_EINVAL", -2: "WC_ENOMEM", -3: "WC_EHIP", -4: "WC_ENOTREADY",
          -5: "WC_ENOCONV", -6: "WC_EBREAKDOWN"}


class WCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("outer_maxit", ctypes.c_int), ("fixed_work", ctypes.c_int), ("check_every", ctypes.c_int),
                ("adjoint", ctypes.c_int), ("use_graph", ctypes.c_int), ("outer", ctypes.c_int),
                ("inner_method", ctypes.c_int), ("persistent", ctypes.c_int)]


OUTER = {"bicgstab": 0, "dc": 1}
INNER_METHOD = {"bicgstab": 0, "pipelined": 1}


class SolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters_total", ctypes.c_int), ("inner_calls", ctypes.c_int),
                ("restarts", ctypes.c_int), ("dslash_count", ctypes.c_long), ("status", ctypes.c_int),
                ("eo_rel_residual", ctypes.c_double), ("true_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("persistent_calls", ctypes.c_int), ("block_size", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def library_path() -> str:
    return _LIBPATH


def load_library():
    """Load libwc.so (built by paper_1709_08785_amd/build.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise ImportError("libwc.so is not built: run `python paper_1709_08785_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(_LIBPATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "wc_solve_params_default": (None, [ctypes.POINTER(SolveParams)]),
        "wc_create_lattice": (I, [ctypes.POINTER(ctypes.c_int), P, ctypes.POINTER(P)]),
        "wc_destroy_lattice": (None, [P]),
        "wc_set_stream": (I, [P, P]),
        "wc_load_links": (I, [P, P]),
        "wc_build_clover": (I, [P, D, D]),
        "wc_set_link_recon": (I, [P, I]),
        "wc_link_recon": (I, [P]),
        "wc_spinor_bytes": (ctypes.c_size_t, [P, I]),
        "wc_pack_spinor": (I, [P, P, P, I]),
        "wc_unpack_spinor": (I, [P, P, P, I]),
        "wc_apply_D": (I, [P, P, P, I]),
        "wc_apply_mult": (I, [P, P, P, I, I]),
        "wc_apply_Dee_oo": (I, [P, P, P, I]),
        "wc_apply_clover": (I, [P, P, P, I, I, I]),
        "wc_solve": (I, [P, P, D, D, D, ctypes.POINTER(SolveParams), P, I, ctypes.POINTER(SolveInfo)]),
        "wc_link_grad": (I, [P, P, P, D, D, I, P]),
        "wc_solve_batch": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(P), D, D, D, ctypes.POINTER(SolveParams),
                               ctypes.POINTER(SolveInfo)]),
        "wc_solve_multi": (I, [I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(D),
                               ctypes.POINTER(D), D, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo)]),
        "wc_set_timing": (I, [P, I]),
        "wc_kernel_slots": (I, []),
        "wc_kernel_stats": (I, [P, I, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_long),
                                ctypes.POINTER(D), ctypes.POINTER(D)]),
        "wc_reset_kernel_stats": (I, [P]),
        "wc_last_error": (ctypes.c_char_p, []),
        "wc_set_barrier_timeout": (I, [D]),
        "wc_set_block_size": (I, [P, I]),
        "wc_link_su3_error": (D, [P]),
        "wc_block_size": (I, [P, I]),
        "wc_tune_block_size": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "wc_set_multi_rhs": (I, [P, I]),
        "wc_set_xcd_chunk": (I, [P, I]),
        "wc_xcd_chunk": (I, [P, I]),
        "wc_set_wave_cap": (I, [P, I, I]),
        "wc_wave_cap": (I, [P, I, I]),
        "wc_set_tune_cache": (I, [ctypes.c_char_p]),
        "wc_apply_Dee_oo_noalloc": (I, [P, P, P, I]),
        "wc_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "wc_apply_mult_batch": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(P), I, I]),
        "wc_apply_Dee_oo_batch": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(P), I]),
        "wc_multi_rhs": (I, [P, I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise WCError(rc, _lib.wc_last_error().decode())


def _prec(p):
    if isinstance(p, str):
        return _PREC_NAMES[p.lower()]
    return int(p)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _require(cond: bool, what: str):
    # argument checks that stay on under python -O (the C ABI takes bare
    # pointers, so a wrong size here would become an access out of bounds)
    if not cond:
        raise ValueError(what)


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


# every open lattice, so that all of them are destroyed while the HIP runtime
# is still fully up: interpreter exit runs these atexit hooks before tearing
# down modules, whereas a lattice left to garbage collection at the very end
# could release its streams, graphs and device memory after the runtime (or a
# profiler attached to it) has begun to unload
_open_lattices = weakref.WeakSet()


@atexit.register
def _close_all_lattices():
    for lat in list(_open_lattices):
        try:
            lat.close()
        except Exception:
            pass


class Lattice:
    """A lattice of extents dims = (Lx, Ly, Lz, Lt) with its links and clover term on the GPU."""

    def __init__(self, dims, device=None):
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.device = torch.device("cuda") if device is None else torch.device(device)
        arr = (ctypes.c_int * 4)(*self.dims)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.wc_create_lattice(arr, self._stream(), ctypes.byref(h)))
        self.h = h
        _open_lattices.add(self)
        lx, ly, lz, lt = self.dims
        self.volume = lx * ly * lz * lt
        self.spinor_shape = (lt, lz, ly, lx, 4, 3)
        self.link_shape = (4, lt, lz, ly, lx, 3, 3)

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        _check(self.lib.wc_set_stream(self.h, self._stream()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.wc_destroy_lattice(self.h)
            self.h = None
        _open_lattices.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _canonical(self, t, name: str, shape=None):
        """t must be a complex128 tensor of the canonical spinor (or given) shape."""
        shape = self.spinor_shape if shape is None else shape
        _require(isinstance(t, torch.Tensor) and t.dtype == torch.complex128 and tuple(t.shape) == shape,
                 "%s must be a complex128 tensor of shape %s" % (name, shape))

    def _eo(self, t, prec, parities: int, name: str):
        """t must hold at least `parities` EO parities in precision prec (any dtype:
        EO fields are raw buffers).  An invalid precision is left to the library,
        which refuses it."""
        p = _prec(prec)
        if p in (FP64, FP32, FP16):
            need = parities * self.spinor_bytes(p)
            _require(isinstance(t, torch.Tensor) and _nbytes(t) >= need,
                     "%s must hold at least %d bytes (%d parity field(s) in precision %d)" % (name, need, parities, p))

    # ---- set-up -------------------------------------------------------------
    def load_links(self, U: torch.Tensor):
        self._canonical(U, "U", self.link_shape)
        self._sync_stream()
        _check(self.lib.wc_load_links(self.h, _ptr(U)))
        self._links_key = None

    def _ensure_links(self, U: torch.Tensor):
        """Load U unless it is the tensor (same storage and version) loaded last."""
        key = (U.data_ptr(), U._version, tuple(U.shape))
        if getattr(self, "_links_key", None) != key:
            self.load_links(U.detach().contiguous())
            self._links_key = key

    def set_link_recon(self, recon: int):
        """Link storage of the FP32 stencil: 12 (two columns), 8 (eight reals) or 18 (full)."""
        self._sync_stream()
        _check(self.lib.wc_set_link_recon(self.h, int(recon)))

    @property
    def link_su3_error(self) -> float:
        """Largest |third column - conj(col0 x col1)| of the loaded links (FP64)."""
        return float(self.lib.wc_link_su3_error(self.h))

    def set_block_size(self, threads: int):
        """Pin the solver kernels' threads per block (64, 128, 256), or 0 to tune."""
        _check(self.lib.wc_set_block_size(self.h, int(threads)))

    def block_size(self, prec=FP32) -> int:
        """Threads per block a solve in this inner precision would use (0: not yet tuned)."""
        return int(self.lib.wc_block_size(self.h, _prec(prec)))

    def tune_block_size(self, prec=FP32) -> dict:
        """Time the inner loop's stencil pair at 64, 128, 256 threads per block and the
        XCD chunks, then the wave caps, and keep the fastest; returns the microseconds per
        pair and the choices."""
        us = (ctypes.c_double * 3)()
        th = ctypes.c_int()
        _check(self.lib.wc_tune_block_size(self.h, _prec(prec), us, ctypes.byref(th)))
        return {"us_per_pair": {64: us[0], 128: us[1], 256: us[2]}, "threads": th.value,
                "chunk": self.xcd_chunk(prec),
                "wave_cap": {"mult": self.wave_cap(prec), "dhat": self.wave_cap(prec, dhat=True)}}

    def set_multi_rhs(self, systems_per_thread: int):
        """Systems per thread of the batched solves' multi-system stencil (2 or 4), 0 for one."""
        _check(self.lib.wc_set_multi_rhs(self.h, int(systems_per_thread)))

    def set_xcd_chunk(self, tiles: int):
        """64-site tiles per XCD chunk of the stencils' workgroup order (0: one slab per XCD,
        -1: tuned with the block size)."""
        _check(self.lib.wc_set_xcd_chunk(self.h, int(tiles)))

    def xcd_chunk(self, prec=FP32) -> int:
        """The XCD chunk a launch in this precision uses now."""
        return int(self.lib.wc_xcd_chunk(self.h, _prec(prec)))

    def set_wave_cap(self, prec, waves_per_cu: int):
        """Pin the one-system stencils in this precision to waves_per_cu waves per CU
        (4, 8, 12, 16; 0: no cap), or -1 to let the tuner choose (default: 8 for FP64,
        none otherwise, before tuning)."""
        _check(self.lib.wc_set_wave_cap(self.h, _prec(prec), int(waves_per_cu)))

    def wave_cap(self, prec=FP64, dhat: bool = False) -> int:
        """The waves-per-CU cap launches in this precision use now, for the D-hat half
        (dhat) or the other stencils (0 = none)."""
        return int(self.lib.wc_wave_cap(self.h, _prec(prec), 1 if dhat else 0))

    def multi_rhs(self, prec=FP32) -> int:
        """Systems per thread of a batched solve's stencil in this precision."""
        return int(self.lib.wc_multi_rhs(self.h, _prec(prec)))

    @property
    def link_recon(self) -> int:
        return int(self.lib.wc_link_recon(self.h))

    def build_clover(self, kappa: float, csw: float):
        self._sync_stream()
        _check(self.lib.wc_build_clover(self.h, float(kappa), float(csw)))

    # ---- EO fields -----------------------------------------------------------
    def spinor_bytes(self, prec) -> int:
        return int(self.lib.wc_spinor_bytes(self.h, _prec(prec)))

    def new_eo(self, prec, parities: int = 1) -> torch.Tensor:
        return torch.zeros(parities * self.spinor_bytes(prec), dtype=torch.uint8, device=self.device)

    def pack(self, psi: torch.Tensor, prec) -> torch.Tensor:
        self._canonical(psi, "psi")
        out = self.new_eo(prec, 2)
        self._sync_stream()
        _check(self.lib.wc_pack_spinor(self.h, _ptr(out), _ptr(psi), _prec(prec)))
        return out

    def unpack(self, eo: torch.Tensor, prec) -> torch.Tensor:
        self._eo(eo, prec, 2, "eo")
        out = torch.empty(self.spinor_shape, dtype=torch.complex128, device=self.device)
        self._sync_stream()
        _check(self.lib.wc_unpack_spinor(self.h, _ptr(out), _ptr(eo), _prec(prec)))
        return out

    def parity_view(self, eo: torch.Tensor, parity: int, prec) -> torch.Tensor:
        sb = self.spinor_bytes(prec)
        return eo[parity * sb:(parity + 1) * sb]

    # ---- operators -------------------------------------------------------------
    def apply_D(self, psi: torch.Tensor, prec=FP64) -> torch.Tensor:
        self._canonical(psi, "psi")
        out = torch.empty_like(psi)
        self._sync_stream()
        _check(self.lib.wc_apply_D(self.h, _ptr(out), _ptr(psi), _prec(prec)))
        return out

    def apply_mult(self, out: torch.Tensor, inp: torch.Tensor, out_parity: int, prec):
        self._eo(out, prec, 1, "out")
        self._eo(inp, prec, 1, "inp")
        self._sync_stream()
        _check(self.lib.wc_apply_mult(self.h, _ptr(out), _ptr(inp), int(out_parity), _prec(prec)))

    def apply_Dee_oo(self, out_e: torch.Tensor, in_e: torch.Tensor, prec):
        self._eo(out_e, prec, 1, "out_e")
        self._eo(in_e, prec, 1, "in_e")
        self._sync_stream()
        _check(self.lib.wc_apply_Dee_oo(self.h, _ptr(out_e), _ptr(in_e), _prec(prec)))

    def apply_Dee_oo_noalloc(self, out_e: torch.Tensor, in_e: torch.Tensor, prec):
        """D-hat_ee with its intermediate in the library's fixed scratch array (no allocation)."""
        self._eo(out_e, prec, 1, "out_e")
        self._eo(in_e, prec, 1, "in_e")
        self._sync_stream()
        _check(self.lib.wc_apply_Dee_oo_noalloc(self.h, _ptr(out_e), _ptr(in_e), _prec(prec)))

    def apply_mult_batch(self, outs, ins, out_parity: int, prec):
        """outs[k] = MULT ins[k] for up to 16 single-parity EO fields, in one launch."""
        n = len(outs)
        _require(len(ins) == n, "outs and ins must have the same length")
        for k in range(n):
            self._eo(outs[k], prec, 1, "outs[%d]" % k)
            self._eo(ins[k], prec, 1, "ins[%d]" % k)
        O = (ctypes.c_void_p * n)(*[_ptr(t).value for t in outs])
        I_ = (ctypes.c_void_p * n)(*[_ptr(t).value for t in ins])
        self._sync_stream()
        _check(self.lib.wc_apply_mult_batch(self.h, n, O, I_, int(out_parity), _prec(prec)))

    def apply_Dee_oo_batch(self, outs, ins, prec):
        """outs[k] = D-hat_ee ins[k] for up to 16 even-parity EO fields."""
        n = len(outs)
        _require(len(ins) == n, "outs and ins must have the same length")
        for k in range(n):
            self._eo(outs[k], prec, 1, "outs[%d]" % k)
            self._eo(ins[k], prec, 1, "ins[%d]" % k)
        O = (ctypes.c_void_p * n)(*[_ptr(t).value for t in outs])
        I_ = (ctypes.c_void_p * n)(*[_ptr(t).value for t in ins])
        self._sync_stream()
        _check(self.lib.wc_apply_Dee_oo_batch(self.h, n, O, I_, _prec(prec)))

    def apply_clover(self, out: torch.Tensor, inp: torch.Tensor, parity: int, inverse: bool, prec):
        self._eo(out, prec, 1, "out")
        self._eo(inp, prec, 1, "inp")
        self._sync_stream()
        _check(self.lib.wc_apply_clover(self.h, _ptr(out), _ptr(inp), int(parity), int(bool(inverse)),
                                        _prec(prec)))

    # ---- solve -------------------------------------------------------------------
    @staticmethod
    def default_params(**kw) -> SolveParams:
        p = SolveParams()
        load_library().wc_solve_params_default(ctypes.byref(p))
        names = {f for f, _ in SolveParams._fields_}
        for k, v in kw.items():
            if k not in names:
                raise TypeError("unknown solver parameter %r" % k)
            if k == "inner_prec":
                v = _prec(v)
            if k == "outer" and isinstance(v, str):
                v = OUTER[v]
            if k == "inner_method" and isinstance(v, str):
                v = INNER_METHOD[v]
            setattr(p, k, v)
        return p

    def solve(self, b: torch.Tensor, kappa: float, csw: float, tol: float, x0: torch.Tensor = None,
              raise_on_error: bool = True, **params):
        """x = D^-1 b; returns (x, info dict).  params go into wc_solve_params."""
        self._canonical(b, "b")
        if x0 is not None:
            self._canonical(x0, "x0")
        p = self.default_params(**params)
        info = SolveInfo()
        x = torch.empty_like(b) if x0 is None else x0.clone()
        self._sync_stream()
        rc = self.lib.wc_solve(self.h, _ptr(b), float(kappa), float(csw), float(tol), ctypes.byref(p), _ptr(x),
                               0 if x0 is None else 1, ctypes.byref(info))
        if rc != 0 and raise_on_error:
            _check(rc)
        d = info.as_dict()
        d["rc"] = rc
        return x, d

    def solve_batch(self, bs, kappa: float, csw: float, tol: float, raise_on_error: bool = True, **params):
        """Solve D x_k = b_k for up to 16 sources together; returns ([x_k], [info_k])."""
        n = len(bs)
        for k, b in enumerate(bs):
            self._canonical(b, "bs[%d]" % k)
        xs = [torch.empty_like(b) for b in bs]
        p = self.default_params(**params)
        infos = (SolveInfo * n)()
        B = (ctypes.c_void_p * n)(*[_ptr(b).value for b in bs])
        X = (ctypes.c_void_p * n)(*[_ptr(x).value for x in xs])
        self._sync_stream()
        rc = self.lib.wc_solve_batch(self.h, n, B, X, float(kappa), float(csw), float(tol), ctypes.byref(p), infos)
        if rc != 0 and raise_on_error:
            _check(rc)
        return xs, [dict(infos[k].as_dict(), rc=rc) for k in range(n)]

    def link_grad(self, lam: torch.Tensor, x: torch.Tensor, kappa: float, csw: float,
                  include_clover: bool = True) -> torch.Tensor:
        """Gradient of -Re<lam, D[U] x> with respect to the loaded links (torch convention)."""
        self._canonical(lam, "lam")
        self._canonical(x, "x")
        G = torch.empty(self.link_shape, dtype=torch.complex128, device=self.device)
        self._sync_stream()
        _check(self.lib.wc_link_grad(self.h, _ptr(lam), _ptr(x), float(kappa), float(csw),
                                     int(bool(include_clover)), _ptr(G)))
        return G

    # ---- timing --------------------------------------------------------------------
    def set_timing(self, on: bool):
        _check(self.lib.wc_set_timing(self.h, int(bool(on))))

    def reset_kernel_stats(self):
        _check(self.lib.wc_reset_kernel_stats(self.h))

    def kernel_stats(self):
        out = {}
        for s in range(self.lib.wc_kernel_slots()):
            name = ctypes.c_char_p()
            n = ctypes.c_long()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            _check(self.lib.wc_kernel_stats(self.h, s, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms),
                                            ctypes.byref(by)))
            out[name.value.decode()] = {"launches": n.value, "ms": ms.value, "bytes": by.value}
        return out


def set_tune_cache(path):
    """File in which the launch-shape tuner keeps its results across processes (None: none)."""
    load_library()
    _check(_lib.wc_set_tune_cache(None if path is None else os.fsencode(path)))


def set_barrier_timeout(seconds: float):
    """Longest wait of a workgroup at a grid barrier of the one-launch inner
    loop (persistent=1) before the solve fails with WC_EHIP; process-wide."""
    load_library()
    _check(_lib.wc_set_barrier_timeout(float(seconds)))


def solve_multi(lats, bs, kappas, csws, tol: float, raise_on_error: bool = True, **params):
    """Solve D_k x_k = b_k on lattices lats[k] (sizes may differ) together, on
    lats[0]'s stream; returns ([x_k], [info_k])."""
    n = len(lats)
    _require(len(bs) == n and len(kappas) == n and len(csws) == n,
             "lats, bs, kappas and csws must have the same length")
    for k in range(n):
        lats[k]._canonical(bs[k], "bs[%d]" % k)
    lib = load_library()
    xs = [torch.empty_like(b) for b in bs]
    p = Lattice.default_params(**params)
    infos = (SolveInfo * n)()
    lats[0]._sync_stream()
    L = (ctypes.c_void_p * n)(*[lat.h.value for lat in lats])
    B = (ctypes.c_void_p * n)(*[_ptr(b).value for b in bs])
    X = (ctypes.c_void_p * n)(*[_ptr(x).value for x in xs])
    K = (ctypes.c_double * n)(*[float(k) for k in kappas])
    C = (ctypes.c_double * n)(*[float(c) for c in csws])
    rc = lib.wc_solve_multi(n, L, B, X, K, C, float(tol), ctypes.byref(p), infos)
    if rc != 0 and raise_on_error:
        _check(rc)
    return xs, [dict(infos[k].as_dict(), rc=rc) for k in range(n)]


class _Solve(torch.autograd.Function):
    """x = D[U]^-1 b with a hand-written backward: the adjoint solve
    lam = D^-dagger g = g5 D^-1 g5 g gives grad_b = lam, and the link gradient
    kernel gives grad_U from (lam, x)."""

    @staticmethod
    def forward(ctx, b, U, lat, kappa, csw, tol, params):
        lat._ensure_links(U)
        x, info = lat.solve(b.detach().contiguous(), kappa, csw, tol, **params)
        ctx.lat, ctx.kappa, ctx.csw, ctx.tol, ctx.params = lat, kappa, csw, tol, params
        ctx.info = info
        ctx.save_for_backward(x, U)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, U = ctx.saved_tensors
        lat = ctx.lat
        lat._ensure_links(U)
        params = dict(ctx.params)
        params["adjoint"] = 1
        lam, _ = lat.solve(gx.detach().contiguous(), ctx.kappa, ctx.csw, ctx.tol, **params)
        gb = lam if ctx.needs_input_grad[0] else None
        gU = lat.link_grad(lam, x, ctx.kappa, ctx.csw) if ctx.needs_input_grad[1] else None
        return gb, gU, None, None, None, None, None


def solve(lat: "Lattice", b: torch.Tensor, U: torch.Tensor, kappa: float, csw: float, tol: float = 1e-10,
          **params) -> torch.Tensor:
    """Differentiable x = D[U]^-1 b (b and U may require grad)."""
    return _Solve.apply(b, U, lat, float(kappa), float(csw), float(tol), params)
