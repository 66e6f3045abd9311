"""Python binding of libkxg (the C ABI declared in include/kxg.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libkxg.so.  Device buffers are torch tensors on a ROCm device
(passed by data pointer), streams are torch streams.  There is no fallback:
if libkxg.so is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; KXG_LIBRARY names another build of the same sources
# (the sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("KXG_LIBRARY") or os.path.join(PKG, "libkxg.so")

# status codes
OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ESTEP, ENUMERIC = range(7)
# precisions
F64, F32, BF16X3, F16X3, F16X2 = 0, 1, 2, 3, 4
PREC_NAMES = {F64: "f64", F32: "f32", BF16X3: "bf16x3", F16X3: "f16x3", F16X2: "f16x2"}
QUAD_GL, QUAD_EXACT = 0, 1
PROJECT = 1
INTERP_LOG = 2
STAT_BOSE = 4
STAT_FERMI = 8
SPLIT_F_ONLY = 16
SPLIT_NONE = 32
WITH_BRACKETS = 1 << 8
LEAN = 1 << 9
NDIAG = 12
NOALLOC_SCRATCH_BYTES = 64 << 20   # the static scratch of kxg_eval_noalloc
RK4, HEUN = 0, 1
EXP_NONE, EXP_RADIATION = 0, 1

EXPORTED = [
    "kxg_kernel_build", "kxg_kernel_free", "kxg_kernel_n", "kxg_kernel_bytes",
    "kxg_kernel_export", "kxg_kernel_grid", "kxg_eval", "kxg_moments",
    "kxg_gauss_legendre", "kxg_stepper_create", "kxg_stepper_free", "kxg_stepper_set",
    "kxg_stepper_release", "kxg_stepper_advance", "kxg_stepper_set_dt",
    "kxg_stepper_query", "kxg_stepper_get", "kxg_stepper_save", "kxg_stepper_load",
    "kxg_last_error", "kxg_profile_begin", "kxg_profile_end", "kxg_kernel_stats",
    "kxg_peak_probe", "kxg_stepper_set_many", "kxg_stepper_bytes", "kxg_eval_noalloc",
]


class KxgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("kxg status %d: %s" % (status, msg))
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.POINTER(ctypes.c_double)),
                ("dp", ctypes.POINTER(ctypes.c_double)), ("mass", ctypes.c_double),
                ("g_dof", ctypes.c_double), ("m2", ctypes.c_double),
                ("n_mu", ctypes.c_int32), ("quad", ctypes.c_int32)]


class KernelInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("packed_blocks", ctypes.c_int64),
                ("nonzero_blocks", ctypes.c_int64), ("gemm_units", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("blocks16", ctypes.c_int64),
                ("nnz_packed", ctypes.c_int64), ("staged16", ctypes.c_int64),
                ("blocks64", ctypes.c_int64), ("blocks_exact", ctypes.c_int64)]


class StepperParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("expansion", ctypes.c_int32), ("project", ctypes.c_int32),
                ("adapt", ctypes.c_int32), ("b_cap", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("atol_rel", ctypes.c_double),
                ("safety", ctypes.c_double), ("fac_min", ctypes.c_double),
                ("fac_max", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("freeze_in", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("h_i", ctypes.c_double),
                ("dt", ctypes.c_double), ("t_end", ctypes.c_double),
                ("max_steps", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("src_n0", ctypes.c_double), ("src_gamma", ctypes.c_double),
                ("src_p0", ctypes.c_double), ("src_kappa", ctypes.c_double),
                ("src_mh", ctypes.c_double), ("src_ti", ctypes.c_double),
                ("du_src", ctypes.c_double), ("eps_switch", ctypes.c_double)]


# keyword names of the freeze-in fields of SolveParams (Stepper.set / set_many)
SOURCE_KEYS = ("src_n0", "src_gamma", "src_p0", "src_kappa", "src_mh", "src_ti", "du_src",
               "eps_switch")


class SlotState(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double),
                ("outflow", ctypes.c_double), ("h_i", ctypes.c_double),
                ("steps", ctypes.c_int32), ("rejected", ctypes.c_int32),
                ("status", ctypes.c_int32), ("phase", ctypes.c_int32),
                ("u_switch", ctypes.c_double), ("n_src", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libkxg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkxg.so not built: run paper_2607_00755_amd/build.py "
                              "(or __graft_entry__.build())")
        # torch first: its HIP runtime is then the one libkxg binds to, so
        # that torch's streams and allocations and the library's calls share
        # one runtime whichever of the two the caller touches first
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.kxg_kernel_build.argtypes = [ctypes.POINTER(Grid), ctypes.c_uint32, ctypes.c_int32,
                                       _vp, ctypes.POINTER(_vp)]
        L.kxg_kernel_free.argtypes = [_vp]
        L.kxg_kernel_free.restype = None
        L.kxg_kernel_n.argtypes = [_vp]
        L.kxg_kernel_bytes.argtypes = [_vp, ctypes.c_int32]
        L.kxg_kernel_bytes.restype = ctypes.c_size_t
        L.kxg_kernel_export.argtypes = [_vp, _dp, _dp]
        L.kxg_kernel_stats.argtypes = [_vp, ctypes.POINTER(KernelInfo)]
        L.kxg_kernel_grid.argtypes = [_vp, _dp, _dp, _dp, _dp]
        L.kxg_eval.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_uint32,
                               _vp, _vp]
        L.kxg_eval_noalloc.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp,
                                       ctypes.c_uint32, _vp, _vp]
        L.kxg_moments.argtypes = [_vp, _vp, ctypes.c_int32, _vp, _vp]
        L.kxg_gauss_legendre.argtypes = [ctypes.c_int32, _dp, _dp]
        L.kxg_stepper_create.argtypes = [_vp, ctypes.POINTER(StepperParams), ctypes.POINTER(_vp)]
        L.kxg_stepper_free.argtypes = [_vp]
        L.kxg_stepper_free.restype = None
        L.kxg_stepper_set.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.POINTER(SolveParams), _vp]
        L.kxg_stepper_set_many.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp,
                                           ctypes.POINTER(SolveParams), _vp]
        L.kxg_stepper_bytes.argtypes = [_vp]
        L.kxg_stepper_bytes.restype = ctypes.c_size_t
        L.kxg_stepper_release.argtypes = [_vp, ctypes.c_int32, _vp]
        L.kxg_stepper_advance.argtypes = [_vp, ctypes.c_int32, _vp]
        L.kxg_stepper_set_dt.argtypes = [_vp, _dp, _vp]
        L.kxg_stepper_query.argtypes = [_vp, ctypes.POINTER(SlotState), _vp]
        L.kxg_stepper_get.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
        L.kxg_stepper_save.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_size_t), _vp]
        L.kxg_stepper_load.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
        L.kxg_profile_begin.argtypes = [ctypes.c_int32]
        L.kxg_profile_end.argtypes = [_dp, ctypes.POINTER(ctypes.c_int32)]
        L.kxg_peak_probe.argtypes = [_dp, _vp]
        L.kxg_last_error.argtypes = []
        L.kxg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().kxg_last_error().decode()


def _check(status: int) -> None:
    if status != OK:
        raise KxgError(status, last_error())


def _stream_ptr(stream) -> Optional[int]:
    """hipStream_t of a torch stream (None -> the current torch stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_ptr(t, n_expected: int, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float64 tensor" % name)
    if t.numel() < n_expected:
        raise ValueError("%s has %d elements, need %d" % (name, t.numel(), n_expected))
    return t.data_ptr()


def profile_begin(capacity: int) -> None:
    """Open a gain-kernel profile (events around each GEMM/stream launch)."""
    _check(lib().kxg_profile_begin(int(capacity)))


def profile_end():
    """Close the profile: (summed kernel milliseconds, launches measured)."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int32(0)
    _check(lib().kxg_profile_end(ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def peak_probe(stream=None) -> dict:
    """kxg_peak_probe: sustained FP32 and BF16 MFMA rates (TFLOP/s), the
    device-memory read bandwidth and the copy bandwidth (GB/s, read +
    written) of this device."""
    out = np.zeros(4)
    _check(lib().kxg_peak_probe(out.ctypes.data_as(_dp), _stream_ptr(stream)))
    return {"mfma_f32_tflops": float(out[0]), "mfma_bf16_tflops": float(out[1]),
            "read_GBps": float(out[2]), "copy_GBps": float(out[3])}


def gauss_legendre(n: int):
    x, w = np.empty(n), np.empty(n)
    _check(lib().kxg_gauss_legendre(n, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp)))
    return x, w


class Kernel:
    """kxg_kernel_build / kxg_eval / kxg_moments / kxg_kernel_export."""

    def __init__(self, p: Sequence[float], precs=(F64,), b_cap: int = 1, mass: float = 1.0,
                 g_dof: float = 1.0, m2: float = 1.0, n_mu: int = 18, quad: int = QUAD_GL,
                 dp: Optional[Sequence[float]] = None, stream=None, brackets: bool = False,
                 lean: bool = False):
        self._h = None
        self.p = np.ascontiguousarray(p, dtype=np.float64)
        self.n = len(self.p)
        self.b_cap = int(b_cap)
        self._dp = None if dp is None else np.ascontiguousarray(dp, dtype=np.float64)
        g = Grid(self.n, self.p.ctypes.data_as(_dp),
                 None if self._dp is None else self._dp.ctypes.data_as(_dp),
                 float(mass), float(g_dof), float(m2), int(n_mu), int(quad))
        mask = (WITH_BRACKETS if brackets else 0) | (LEAN if lean else 0)
        for q in precs:
            mask |= 1 << int(q)
        h = _vp()
        st = None if stream is None and not _cuda_ready() else _stream_ptr(stream)
        _check(lib().kxg_kernel_build(ctypes.byref(g), mask, self.b_cap, st, ctypes.byref(h)))
        self._h = h
        self.precs = tuple(precs)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kxg_kernel_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def bytes(self, prec: int = -1) -> int:
        return int(lib().kxg_kernel_bytes(self._h, prec))

    def stats(self) -> dict:
        """kxg_kernel_stats: blocks of the packed operand, kept blocks, units."""
        info = KernelInfo()
        _check(lib().kxg_kernel_stats(self._h, ctypes.byref(info)))
        return {"n": info.n, "packed_blocks": info.packed_blocks,
                "nonzero_blocks": info.nonzero_blocks, "gemm_units": info.gemm_units,
                "max_slots": info.max_slots, "blocks16": info.blocks16,
                "nnz_packed": info.nnz_packed, "staged16": info.staged16,
                "blocks64": info.blocks64, "blocks_exact": info.blocks_exact}

    def export(self):
        n = self.n
        A = np.empty((n, n, n))
        R = np.empty((n, n))
        _check(lib().kxg_kernel_export(self._h, A.ctypes.data_as(_dp), R.ctypes.data_as(_dp)))
        return A, R

    def grid(self):
        out = [np.empty(self.n) for _ in range(4)]
        _check(lib().kxg_kernel_grid(self._h, *(a.ctypes.data_as(_dp) for a in out)))
        return dict(zip(("dp", "E", "K", "h"), out))

    def eval(self, f, prec: int = F64, project: bool = True, out=None, diag=None, stream=None,
             log_interp: bool = False, eta: int = 0, diagnostics: bool = True, split: int = 3):
        """C[f] for f of shape [B, n] (device float64).  Returns (C, diag).
        log_interp / eta (+1 Bose-Einstein, -1 Fermi-Dirac) select the exact
        form of the operator (handle built with brackets=True).  With
        diagnostics=False no diagnostics are computed and diag is None.
        split (16-bit precisions): 3 products of the hi+lo split (default), 2
        (F2 split only) or 1 (no split), the latter two as ablations."""
        return self._eval(lib().kxg_eval, f, prec, project, out, diag, stream, log_interp,
                          eta, diagnostics, split)

    def eval_noalloc(self, f, prec: int = F64, project: bool = True, out=None, diag=None,
                     stream=None, log_interp: bool = False, eta: int = 0,
                     diagnostics: bool = True, split: int = 3):
        """eval through kxg_eval_noalloc: the same result, with the call's
        workspace in the library's static device array (raises KxgError when
        the call needs more than that array holds)."""
        return self._eval(lib().kxg_eval_noalloc, f, prec, project, out, diag, stream,
                          log_interp, eta, diagnostics, split)

    def _eval(self, entry, f, prec, project, out, diag, stream, log_interp, eta, diagnostics,
              split):
        import torch
        if f.dim() == 1:
            f = f.view(1, -1)
        B = f.shape[0]
        if out is None:
            out = torch.empty_like(f)
        if diag is None and diagnostics:
            diag = torch.empty((B, NDIAG), dtype=torch.float64, device=f.device)
        flags = (PROJECT if project else 0) | (INTERP_LOG if log_interp else 0)
        flags |= STAT_BOSE if eta > 0 else (STAT_FERMI if eta < 0 else 0)
        flags |= {3: 0, 2: SPLIT_F_ONLY, 1: SPLIT_NONE}[split]
        _check(entry(self._h, int(prec), _dev_ptr(f, B * self.n, "f"), B,
                     _dev_ptr(out, B * self.n, "C"), flags,
                     _dev_ptr(diag, B * NDIAG, "diag") if diag is not None else None,
                     _stream_ptr(stream)))
        return out, diag

    def moments(self, f, out=None, stream=None):
        import torch
        if f.dim() == 1:
            f = f.view(1, -1)
        B = f.shape[0]
        if out is None:
            out = torch.empty((B, 3), dtype=torch.float64, device=f.device)
        _check(lib().kxg_moments(self._h, _dev_ptr(f, B * self.n, "f"), B,
                                 _dev_ptr(out, 3 * B, "out"), _stream_ptr(stream)))
        return out


def _cuda_ready() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _solve_params(lam, h_i, dt, t_end, max_steps, sources) -> SolveParams:
    bad = set(sources) - set(SOURCE_KEYS)
    if bad:
        raise TypeError("unknown solve parameters: %s" % sorted(bad))
    sp = SolveParams(float(lam), float(h_i), float(dt), float(t_end), int(max_steps), 0)
    for k, v in sources.items():
        setattr(sp, k, float(v))
    return sp


class Stepper:
    """kxg_stepper_*: on-device RK4 / adaptive Heun over many slots."""

    def __init__(self, kernel: Kernel, kind: int = RK4, prec: int = F64, b_cap: int = 1,
                 expansion: int = EXP_NONE, project: bool = True, adapt: bool = True,
                 rtol: float = 1e-6, atol_rel: float = 1e-12, safety: float = 0.9,
                 fac_min: float = 0.2, fac_max: float = 5.0, dt_min: float = 1e-14,
                 freeze_in: bool = False):
        self._h = None
        self.kernel = kernel
        self.n = kernel.n
        self.b_cap = int(b_cap)
        self.expansion = int(expansion)
        prm = StepperParams(int(kind), int(prec), int(expansion), int(bool(project)),
                            int(bool(adapt)), self.b_cap, rtol, atol_rel, safety, fac_min,
                            fac_max, dt_min, int(bool(freeze_in)), 0)
        h = _vp()
        _check(lib().kxg_stepper_create(kernel.handle, ctypes.byref(prm), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kxg_stepper_free(self._h)
            self._h = None

    def set(self, slot: int, f0, lam: float, t_end: float, dt: float = 0.0, h_i: float = 0.0,
            max_steps: int = 0, stream=None, **sources):
        """Load one slot; freeze-in keywords (SOURCE_KEYS) set the sources
        and the source-only regime of steppers created with freeze_in."""
        sp = _solve_params(lam, h_i, dt, t_end, max_steps, sources)
        _check(lib().kxg_stepper_set(self._h, int(slot), _dev_ptr(f0, self.n, "f0"),
                                     ctypes.byref(sp), _stream_ptr(stream)))

    def set_many(self, slot0: int, f0, lam, t_end, dt=0.0, h_i=0.0, max_steps=0, stream=None,
                 **sources):
        """Load slots slot0 .. slot0 + len(f0) - 1 in one call (f0: device
        [count, n] float64; the other arguments, freeze-in keywords included,
        are scalars or one value per slot)."""
        count = f0.shape[0] if f0.dim() == 2 else 1
        per = lambda v: np.broadcast_to(np.asarray(v, dtype=np.float64), (count,))
        lam_, te_, dt_, hi_ = per(lam), per(t_end), per(dt), per(h_i)
        ms_ = np.broadcast_to(np.asarray(max_steps, dtype=np.int64), (count,))
        src_ = {k: per(v) for k, v in sources.items()}
        arr = (SolveParams * count)()
        for j in range(count):
            arr[j] = _solve_params(lam_[j], hi_[j], dt_[j], te_[j], ms_[j],
                                   {k: v[j] for k, v in src_.items()})
        _check(lib().kxg_stepper_set_many(self._h, int(slot0), int(count),
                                          _dev_ptr(f0, count * self.n, "f0"), arr,
                                          _stream_ptr(stream)))

    def bytes(self) -> int:
        """Device bytes the stepper holds."""
        return int(lib().kxg_stepper_bytes(self._h))

    def release(self, slot: int, stream=None):
        _check(lib().kxg_stepper_release(self._h, int(slot), _stream_ptr(stream)))

    def advance(self, n_iter: int = 1, stream=None):
        _check(lib().kxg_stepper_advance(self._h, int(n_iter), _stream_ptr(stream)))

    def set_dt(self, dt: Sequence[float], stream=None):
        a = np.ascontiguousarray(dt, dtype=np.float64)
        if a.size != self.b_cap:
            raise ValueError("need one dt per slot")
        _check(lib().kxg_stepper_set_dt(self._h, a.ctypes.data_as(_dp), _stream_ptr(stream)))

    def query(self, stream=None):
        arr = (SlotState * self.b_cap)()
        _check(lib().kxg_stepper_query(self._h, arr, _stream_ptr(stream)))
        return [{"t": s.t, "dt": s.dt, "outflow": s.outflow, "h_i": s.h_i, "steps": s.steps,
                 "rejected": s.rejected, "status": s.status, "phase": s.phase,
                 "u_switch": s.u_switch, "n_src": s.n_src} for s in arr]

    def get(self, slot: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(lib().kxg_stepper_get(self._h, int(slot), _dev_ptr(out, self.n, "out"),
                                     _stream_ptr(stream)))
        return out

    def save(self, slot: int, stream=None) -> bytes:
        ln = ctypes.c_size_t(0)
        _check(lib().kxg_stepper_save(self._h, int(slot), None, ctypes.byref(ln), _stream_ptr(stream)))
        buf = ctypes.create_string_buffer(ln.value)
        _check(lib().kxg_stepper_save(self._h, int(slot), buf, ctypes.byref(ln), _stream_ptr(stream)))
        return buf.raw[: ln.value]

    def load(self, slot: int, blob: bytes, stream=None):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().kxg_stepper_load(self._h, int(slot), buf, len(blob), _stream_ptr(stream)))
