"""Python binding of the SFFT gfx950 library (``libsfft.so``).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels. PyTorch provides device memory (tensors) and streams. The
binding refuses to run when the library has not been built -- there is no
CPU fallback.

The names mirror the C ABI of ``include/sfft.h``: ``build_system``,
``solve``, ``subtract``, ``run``, ``submit`` / ``poll`` / ``wait``.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfft.so")

OK, PENDING = 0, 1
E_INVAL, E_NOMEM, E_NOT_SPD, E_NONFINITE, E_UNSUPPORTED, E_HIP, E_NOTFOUND = -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
F32, F64 = 0, 1

_lib = None
_lib_lock = threading.Lock()


class SfftError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = lib().sfft_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class _Params(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int32), ("n1", ctypes.c_int32), ("w0", ctypes.c_int32),
                ("w1", ctypes.c_int32), ("dk", ctypes.c_int32), ("db", ctypes.c_int32),
                ("const_phot_ratio", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dtype", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("p", _Params), ("r_fit", ctypes.c_void_p), ("s_fit", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


@dataclass(frozen=True)
class Params:
    """Problem parameters: image shape (n0, n1), kernel half widths (w0, w1),
    kernel / background polynomial degrees (dk, db), ConstPhotRatio flag,
    arithmetic (FP64 or MIXED) and image element type (F32 or F64)."""

    n0: int
    n1: int
    w0: int
    w1: int
    dk: int
    db: int
    const_phot: int = 0
    precision: int = MIXED
    dtype: int = F32

    def c(self) -> _Params:
        return _Params(self.n0, self.n1, self.w0, self.w1, self.dk, self.db, self.const_phot,
                       self.precision, self.dtype)

    @property
    def torch_dtype(self):
        return torch.float32 if self.dtype == F32 else torch.float64

    @property
    def num_unknowns(self) -> int:
        return int(lib().sfft_num_unknowns(ctypes.byref(self.c())))


def lib():
    """Load ``libsfft.so`` (after torch, so both share one HIP runtime)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2109_09334_amd.build`; there is no fallback")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
            pp = ctypes.POINTER(_Params)
            L.sfft_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_size_t]
            L.sfft_destroy.argtypes = [vp]
            L.sfft_destroy.restype = None
            L.sfft_num_unknowns.argtypes = [pp]
            L.sfft_num_unknowns.restype = i64
            L.sfft_check_params.argtypes = [pp]
            L.sfft_workspace_bytes.argtypes = [pp]
            L.sfft_workspace_bytes.restype = i64
            L.sfft_build_system.argtypes = [vp, pp, vp, vp, vp, vp, vp]
            L.sfft_solve.argtypes = [vp, pp, vp, vp, vp, vp, vp, vp]
            L.sfft_subtract.argtypes = [vp, pp, vp, vp, vp, vp, vp]
            L.sfft_run.argtypes = [vp, pp, vp, vp, vp, vp, vp, vp, vp]
            L.sfft_run_noalloc.argtypes = [vp, pp, vp, vp, vp, vp, vp, vp, vp]
            L.sfft_run_batch.argtypes = [vp, ctypes.POINTER(_Request), i32, vp]
            dbl = ctypes.c_double
            L.sfft_decorrelate.argtypes = [vp, pp, vp, dbl, dbl, i32, vp, vp, i32, vp, vp, vp, vp, vp]
            L.sfft_crowded_mask.argtypes = [vp, i32, i32, i32, vp, vp, dbl, dbl, i32, i32, i32, i32,
                                            vp, vp, vp, vp]
            L.sfft_sync.argtypes = [vp, vp]
            L.sfft_lag_tables.argtypes = [vp, pp, vp, vp, vp, vp, vp, vp, vp, vp]
            L.sfft_fft_lines.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp]
            L.sfft_engine_config.argtypes = [vp, i32, i32]
            L.sfft_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
            L.sfft_poll.argtypes = [vp, ctypes.c_uint64]
            L.sfft_wait.argtypes = [vp, ctypes.c_uint64]
            L.sfft_profile.argtypes = [vp, i32]
            L.sfft_debug_solve_stall.argtypes = [vp, i32]
            L.sfft_profile_read.argtypes = [vp, i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int)]
            L.sfft_strerror.argtypes = [i32]
            L.sfft_strerror.restype = ctypes.c_char_p
            for name in ("sfft_create", "sfft_check_params", "sfft_build_system", "sfft_solve",
                         "sfft_subtract", "sfft_run", "sfft_run_noalloc", "sfft_run_batch", "sfft_decorrelate",
                         "sfft_crowded_mask",
                         "sfft_sync",
                         "sfft_lag_tables",
                         "sfft_fft_lines", "sfft_engine_config", "sfft_profile", "sfft_profile_read", "sfft_submit", "sfft_poll",
                         "sfft_wait", "sfft_debug_solve_stall"):
                getattr(L, name).restype = i32
            _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc not in (OK, PENDING):
        raise SfftError(rc, what)
    return rc


def _ptr(t: torch.Tensor | None, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One library context on a device: plans, workspaces, serving engine."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        torch.cuda.init()
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().sfft_create(ctypes.byref(h), device, hbm_budget_bytes), "sfft_create")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().sfft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- validation helpers -------------------------------------------------
    @staticmethod
    def check(p: Params) -> int:
        return int(lib().sfft_check_params(ctypes.byref(p.c())))

    @staticmethod
    def workspace_bytes(p: Params) -> int:
        return int(lib().sfft_workspace_bytes(ctypes.byref(p.c())))

    def _img(self, p: Params, t, name):
        return _ptr(t, p.torch_dtype, p.n0 * p.n1, name)

    # -- hot path -----------------------------------------------------------
    def build_system(self, p: Params, r_fit, s_fit, stream=None):
        n = p.num_unknowns
        dev = r_fit.device
        G = torch.empty((n, n), dtype=torch.float64, device=dev)
        h = torch.empty(n, dtype=torch.float64, device=dev)
        _check(lib().sfft_build_system(self._h, ctypes.byref(p.c()), self._img(p, r_fit, "r_fit"),
                                       self._img(p, s_fit, "s_fit"), _ptr(G), _ptr(h),
                                       _stream(stream)), "sfft_build_system")
        return G, h

    def solve(self, p: Params, G, h, r_fit=None, s_fit=None, stream=None, sync=True):
        """On the null stream (torch's default) the C call is itself
        synchronous and raises NOT_SPD / NONFINITE directly."""
        n = p.num_unknowns
        coef = torch.empty(n, dtype=torch.float64, device=G.device)
        _check(lib().sfft_solve(self._h, ctypes.byref(p.c()), _ptr(G, torch.float64, n * n, "G"),
                                _ptr(h, torch.float64, n, "h"), self._img(p, r_fit, "r_fit"),
                                self._img(p, s_fit, "s_fit"), _ptr(coef), _stream(stream)),
               "sfft_solve")
        if sync:
            self.sync(stream)
        return coef

    def subtract(self, p: Params, r, s, coef, stream=None):
        d = torch.empty((p.n0, p.n1), dtype=p.torch_dtype, device=r.device)
        _check(lib().sfft_subtract(self._h, ctypes.byref(p.c()), self._img(p, r, "r"),
                                   self._img(p, s, "s"),
                                   _ptr(coef, torch.float64, p.num_unknowns, "coef"), _ptr(d),
                                   _stream(stream)), "sfft_subtract")
        return d

    def run(self, p: Params, r_fit, s_fit, r=None, s=None, coef=None, d=None, stream=None):
        r = r_fit if r is None else r
        s = s_fit if s is None else s
        if coef is None:
            coef = torch.empty(p.num_unknowns, dtype=torch.float64, device=r.device)
        if d is None:
            d = torch.empty((p.n0, p.n1), dtype=p.torch_dtype, device=r.device)
        _check(lib().sfft_run(self._h, ctypes.byref(p.c()), self._img(p, r_fit, "r_fit"),
                              self._img(p, s_fit, "s_fit"), self._img(p, r, "r"),
                              self._img(p, s, "s"),
                              _ptr(coef, torch.float64, p.num_unknowns, "coef"),
                              self._img(p, d, "d"), _stream(stream)), "sfft_run")
        return coef, d

    def run_batch(self, p: Params, items, stream=None):
        """sfft_run_batch: items = [(r_fit, s_fit, r, s, coef or None, d)],
        all of variant p, as one launch per stage."""
        n = len(items)
        arr = (_Request * n)()
        for z, (rf, sf, r, s, coef, d) in enumerate(items):
            arr[z] = _Request(p.c(), self._img(p, rf, "r_fit"), self._img(p, sf, "s_fit"),
                              self._img(p, r, "r"), self._img(p, s, "s"),
                              _ptr(coef, torch.float64, p.num_unknowns, "coef") if coef is not None
                              else None, self._img(p, d, "d"), None)
        _check(lib().sfft_run_batch(self._h, arr, n, _stream(stream)), "sfft_run_batch")

    def run_noalloc(self, p: Params, r_fit, s_fit, r=None, s=None, coef=None, d=None,
                    stream=None):
        """sfft_run_noalloc: the library allocates nothing (outputs are the
        caller's; created here only when not given)."""
        r = r_fit if r is None else r
        s = s_fit if s is None else s
        if d is None:
            d = torch.empty((p.n0, p.n1), dtype=p.torch_dtype, device=r.device)
        _check(lib().sfft_run_noalloc(self._h, ctypes.byref(p.c()), self._img(p, r_fit, "r_fit"),
                                      self._img(p, s_fit, "s_fit"), self._img(p, r, "r"),
                                      self._img(p, s, "s"),
                                      None if coef is None else
                                      _ptr(coef, torch.float64, p.num_unknowns, "coef"),
                                      self._img(p, d, "d"), _stream(stream)), "sfft_run_noalloc")
        return coef, d

    def decorrelate(self, p: Params, coef, d, u0: float, u1: float, sigma_sci, sigma_ref,
                    g_sci=None, h_ref=None, out=None, stream=None):
        """sfft_decorrelate: d (x) Q (App. C). sigma_sci, sigma_ref: FP64
        device vectors (one entry per co-added image); g_sci, h_ref: FP64
        device stamps [count][2 w0 + 1][2 w1 + 1] or None (unit stamps)."""
        if out is None:
            out = torch.empty((p.n0, p.n1), dtype=p.torch_dtype, device=d.device)
        m, n = sigma_sci.numel(), sigma_ref.numel()
        L = (2 * p.w0 + 1) * (2 * p.w1 + 1)
        _check(lib().sfft_decorrelate(
            self._h, ctypes.byref(p.c()), _ptr(coef, torch.float64, p.num_unknowns, "coef"),
            float(u0), float(u1), m, _ptr(sigma_sci, torch.float64, None, "sigma_sci"),
            _ptr(g_sci, torch.float64, m * L, "g_sci"), n,
            _ptr(sigma_ref, torch.float64, None, "sigma_ref"),
            _ptr(h_ref, torch.float64, n * L, "h_ref"), self._img(p, d, "d"),
            self._img(p, out, "out"), _stream(stream)), "sfft_decorrelate")
        return out

    def crowded_mask(self, r, s, u_r: float, u_s: float, g0: int, g1: int, t0: int = 64,
                     t1: int = 64, r_out=None, s_out=None, want_mask: bool = False, stream=None):
        """sfft_crowded_mask (Sec. 3.1): the masked fit pair (r_out, s_out)
        and, with want_mask, the uint8 mask."""
        if r.dtype not in (torch.float32, torch.float64) or s.dtype != r.dtype or r.shape != s.shape:
            raise ValueError("r, s must be images of one shape and type (float32 or float64)")
        n0, n1 = r.shape
        r_out = torch.empty_like(r) if r_out is None else r_out
        s_out = torch.empty_like(s) if s_out is None else s_out
        m = torch.empty((n0, n1), dtype=torch.uint8, device=r.device) if want_mask else None
        for t, nm in ((r, "r"), (s, "s"), (r_out, "r_out"), (s_out, "s_out")):
            _ptr(t, r.dtype, n0 * n1, nm)
        _check(lib().sfft_crowded_mask(self._h, n0, n1, F32 if r.dtype == torch.float32 else F64,
                                       _ptr(r), _ptr(s), float(u_r), float(u_s), g0, g1, t0, t1,
                                       _ptr(r_out), _ptr(s_out), _ptr(m, torch.uint8),
                                       _stream(stream)), "sfft_crowded_mask")
        return (r_out, s_out, m) if want_mask else (r_out, s_out)

    def sync(self, stream=None):
        _check(lib().sfft_sync(self._h, _stream(stream)), "sfft_sync")

    def lag_tables(self, p: Params, r_fit, s_fit, stream=None):
        P = (p.dk + 1) * (p.dk + 2) // 2
        Q = (p.db + 1) * (p.db + 2) // 2
        dev = r_fit.device
        f64 = dict(dtype=torch.float64, device=dev)
        om = torch.empty((P * (P + 1) // 2, 4 * p.w0 + 1, 4 * p.w1 + 1), **f64)
        th = torch.empty((P, 2 * p.w0 + 1, 2 * p.w1 + 1), **f64)
        la = torch.empty((P, Q, 2 * p.w0 + 1, 2 * p.w1 + 1), **f64)
        cm = torch.empty((Q, Q), **f64)
        ev = torch.empty(Q, **f64)
        _check(lib().sfft_lag_tables(self._h, ctypes.byref(p.c()), self._img(p, r_fit, "r_fit"),
                                     self._img(p, s_fit, "s_fit"), _ptr(om), _ptr(th), _ptr(la),
                                     _ptr(cm), _ptr(ev), _stream(stream)), "sfft_lag_tables")
        return {"omega": om, "theta": th, "lambda": la, "cmat": cm, "evec": ev}

    def fft_lines(self, x: torch.Tensor, sign: int = -1, stream=None):
        """Transform the last axis of a complex64/complex128 tensor."""
        if x.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("complex64 or complex128 expected")
        x = x.contiguous()
        out = torch.empty_like(x)
        n = x.shape[-1]
        lines = x.numel() // n
        dt = F32 if x.dtype == torch.complex64 else F64
        _check(lib().sfft_fft_lines(self._h, n, lines, sign, dt, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "sfft_fft_lines")
        return out

    # -- stage timers ---------------------------------------------------------
    def profile(self, enable: bool = True):
        _check(lib().sfft_profile(self._h, 1 if enable else 0), "sfft_profile")

    def profile_read(self) -> dict:
        """{stage: (total_ms, calls)} for the direct calls since profile()."""
        cap = 64
        names = ctypes.create_string_buffer(32 * cap)
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int * cap)()
        n = lib().sfft_profile_read(self._h, cap, names, ms, cnt)
        if n < 0:
            raise SfftError(n, "sfft_profile_read")
        out = {}
        for i in range(min(n, cap)):
            nm = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (ms[i], cnt[i])
        return out

    # -- serving engine -----------------------------------------------------
    def engine_config(self, slots: int = 4, max_batch: int = 4):
        _check(lib().sfft_engine_config(self._h, slots, max_batch), "sfft_engine_config")

    def debug_solve_stall(self, enable: bool = True):
        """Make the triangular solves' bounded waits give up (diagnostics)."""
        _check(lib().sfft_debug_solve_stall(self._h, 1 if enable else 0), "sfft_debug_solve_stall")

    def submit(self, p: Params, r_fit, s_fit, r, s, coef, d, stream=None) -> int:
        """Queue one request. It starts after the work already enqueued on
        `stream` (torch's current stream by default); its tensors are held
        here until poll/wait has returned its final status."""
        req = _Request(p.c(), self._img(p, r_fit, "r_fit"), self._img(p, s_fit, "s_fit"),
                       self._img(p, r, "r"), self._img(p, s, "s"),
                       _ptr(coef, torch.float64, p.num_unknowns, "coef") if coef is not None else None,
                       self._img(p, d, "d"), _stream(stream))
        t = ctypes.c_uint64()
        _check(lib().sfft_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "sfft_submit")
        self._keep[t.value] = (r_fit, s_fit, r, s, coef, d)
        return t.value

    def poll(self, ticket: int) -> int:
        rc = lib().sfft_poll(self._h, ticket)
        if rc != PENDING:
            self._keep.pop(ticket, None)
        if rc not in (OK, PENDING):
            raise SfftError(rc, f"request {ticket}")
        return rc

    def wait(self, ticket: int) -> int:
        rc = lib().sfft_wait(self._h, ticket)
        self._keep.pop(ticket, None)
        if rc != OK:
            raise SfftError(rc, f"request {ticket}")
        return rc


def num_unknowns(w0, w1, dk, db, const_phot=0) -> int:
    return int(lib().sfft_num_unknowns(ctypes.byref(_Params(16, 16, w0, w1, dk, db, const_phot, 0, 0))))


def strerror(code: int) -> str:
    return lib().sfft_strerror(code).decode()
