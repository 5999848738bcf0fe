"""Python binding of libmp.so (include/mp.h): argument marshalling only.

Every step of the decode runs in the library's HIP kernels; this module only
turns torch device tensors into pointers and sizes, and status codes into
exceptions.  If libmp.so is missing it raises at import time -- there is no
fallback.

Low level: :func:`mp_create`, :func:`mp_solve`, :func:`mp_destroy`, ... with
the C names.  High level: :class:`Decoder`.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mp.h")

MP_OK, MP_EINVAL, MP_ENOTNORM, MP_ENONFINITE, MP_ENOMEM, MP_EDEVICE, MP_EUNSUPPORTED = range(7)
MP_F32, MP_BF16, MP_FP8_E4M3, MP_F64, MP_SIGN1 = 0, 1, 2, 3, 4
STOP_CONVERGED, STOP_MAX_ITERS, STOP_STALLED, STOP_ZERO_INPUT = 0, 1, 2, 3
STOP_NAMES = {0: "converged", 1: "max_iters", 2: "stalled", 3: "zero_input"}
MP_SKIP_NORM_CHECK = 0x1
MP_SOLVE_STEP_LAUNCHES = 0x1  # mp_opts.flags
MP_SOLVE_ASYNC = 0x2  # mp_opts.flags
DTYPES = {"f32": MP_F32, "bf16": MP_BF16, "fp8": MP_FP8_E4M3, "f64": MP_F64, "sign": MP_SIGN1}


class Opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("max_iters", ctypes.c_int64),
                ("rescore_k", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("yy", ctypes.c_double), ("rr", ctypes.c_double),
                ("stop_reason", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class Trace(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("rr", ctypes.c_void_p),
                ("cap", ctypes.c_int64), ("r", ctypes.c_void_p), ("ldr", ctypes.c_int64)]


class TraceF64(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("rr", ctypes.c_void_p),
                ("cap", ctypes.c_int64), ("r", ctypes.c_void_p), ("ldr", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_void_p), ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("ld", ctypes.c_int64)]


class RaggedConfig(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("cols_per_wave", ctypes.c_int32),
                ("wgs_per_cu", ctypes.c_int32), ("split", ctypes.c_int32)]


class BatchedConfig(ctypes.Structure):
    _fields_ = [("atoms128_above", ctypes.c_int32), ("atoms64_above", ctypes.c_int32),
                ("atoms32_above", ctypes.c_int32)]


class MPError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {_status_str(status)}: {detail}")


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_0809_1833_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, u32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32
    lib.mp_create.restype = ctypes.c_int
    lib.mp_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), p, i64, i64, i64, ctypes.c_int,
                              u32, p]
    lib.mp_solve.restype = ctypes.c_int
    lib.mp_solve.argtypes = [p, p, p, p, ctypes.POINTER(Opts), ctypes.POINTER(Result),
                             ctypes.POINTER(Trace), p]
    lib.mp_solve_result.restype = ctypes.c_int
    lib.mp_solve_result.argtypes = [p, ctypes.POINTER(Result)]
    lib.mp_solve_noalloc.restype = ctypes.c_int
    lib.mp_solve_noalloc.argtypes = [p, p, p, p, ctypes.POINTER(Opts), ctypes.POINTER(Result),
                                     ctypes.POINTER(Trace), p]
    lib.mp_destroy.restype = None
    lib.mp_destroy.argtypes = [p]
    lib.mp_status_str.restype = ctypes.c_char_p
    lib.mp_status_str.argtypes = [ctypes.c_int]
    lib.mp_last_error.restype = ctypes.c_char_p
    lib.mp_last_error.argtypes = [p]
    lib.mp_solve_batched.restype = ctypes.c_int
    lib.mp_solve_batched.argtypes = [p, p, i64, i64, p, i64, p, i64, ctypes.POINTER(Opts), p,
                                     p, ctypes.POINTER(Trace), p]
    lib.mp_create_ragged.restype = ctypes.c_int
    lib.mp_create_ragged.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Instance),
                                     i64, ctypes.c_int, u32, p]
    lib.mp_solve_ragged.restype = ctypes.c_int
    lib.mp_solve_ragged.argtypes = [p, p, p, p, ctypes.POINTER(Opts), p, p,
                                    ctypes.POINTER(Trace), p]
    lib.mp_batched_set_config.restype = ctypes.c_int
    lib.mp_batched_set_config.argtypes = [p, ctypes.POINTER(BatchedConfig)]
    lib.mp_batched_get_config.restype = ctypes.c_int
    lib.mp_batched_get_config.argtypes = [p, ctypes.POINTER(BatchedConfig)]
    lib.mp_ragged_set_config.restype = ctypes.c_int
    lib.mp_ragged_set_config.argtypes = [p, ctypes.POINTER(RaggedConfig)]
    lib.mp_ragged_get_config.restype = ctypes.c_int
    lib.mp_ragged_get_config.argtypes = [p, ctypes.POINTER(RaggedConfig)]
    lib.mp_get_storage.restype = ctypes.c_int
    lib.mp_get_storage.argtypes = [p, p, p, p]
    lib.mp_set_profiling.restype = ctypes.c_int
    lib.mp_set_profiling.argtypes = [p, ctypes.c_int]
    lib.mp_kernel_time.restype = ctypes.c_int
    lib.mp_kernel_time.argtypes = [p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.mp_solve_omp.restype = ctypes.c_int
    lib.mp_solve_omp.argtypes = [p, p, p, p, ctypes.POINTER(Opts), ctypes.POINTER(Result),
                                 ctypes.POINTER(Trace), p]
    lib.mp_create_f64.restype = ctypes.c_int
    lib.mp_create_f64.argtypes = [ctypes.POINTER(ctypes.c_void_p), p, i64, i64, i64, u32, p]
    lib.mp_create_signs.restype = ctypes.c_int
    lib.mp_create_signs.argtypes = [ctypes.POINTER(ctypes.c_void_p), p, i64, i64, i64, u32, p]
    lib.mp_solve_f64.restype = ctypes.c_int
    lib.mp_solve_f64.argtypes = [p, p, p, p, ctypes.POINTER(Opts), ctypes.POINTER(Result),
                                 ctypes.POINTER(TraceF64), p]
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises if libmp.so is not built)."""
    return _load()


def header_functions(path: str = HEADER):
    """Names of the functions include/mp.h declares."""
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(mp_\w+)\s*\(", text, flags=re.M)))


def _status_str(s: int) -> str:
    try:
        return _load().mp_status_str(int(s)).decode()
    except Exception:  # pragma: no cover - library missing
        return str(s)


def _check(status: int, where: str, ctx=None):
    if status != MP_OK:
        detail = _load().mp_last_error(ctx).decode(errors="replace")
        raise MPError(status, where, detail)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---- C-named wrappers --------------------------------------------------------

def mp_create(psi_ptr: int, n: int, m: int, ld: int, storage: int = MP_F32, flags: int = 0,
              stream: Optional[int] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = _load().mp_create(ctypes.byref(h), psi_ptr, n, m, ld, storage, flags, stream)
    _check(st, "mp_create", None)
    return h


def mp_solve(ctx, y_ptr: int, x_ptr: int, r_ptr: Optional[int], opts: Opts,
             trace: Optional[Trace] = None, stream: Optional[int] = None,
             want_result: bool = True) -> Optional[Result]:
    """``want_result=False`` passes res = NULL (required with MP_SOLVE_ASYNC)."""
    res = Result() if want_result else None
    st = _load().mp_solve(ctx, y_ptr, x_ptr, r_ptr, ctypes.byref(opts),
                          ctypes.byref(res) if res is not None else None,
                          ctypes.byref(trace) if trace is not None else None, stream)
    _check(st, "mp_solve", ctx)
    return res


def mp_solve_noalloc(ctx, y_ptr: int, x_ptr: int, r_ptr: Optional[int], opts: Opts,
                     trace: Optional[Trace] = None, stream: Optional[int] = None,
                     want_result: bool = True) -> Optional[Result]:
    res = Result() if want_result else None
    st = _load().mp_solve_noalloc(ctx, y_ptr, x_ptr, r_ptr, ctypes.byref(opts),
                                  ctypes.byref(res) if res is not None else None,
                                  ctypes.byref(trace) if trace is not None else None, stream)
    _check(st, "mp_solve_noalloc", ctx)
    return res


def mp_solve_result(ctx) -> Result:
    res = Result()
    _check(_load().mp_solve_result(ctx, ctypes.byref(res)), "mp_solve_result", ctx)
    return res


def mp_solve_omp(ctx, y_ptr: int, x_ptr: int, r_ptr: Optional[int], opts: Opts,
                 trace: Optional[Trace] = None, stream: Optional[int] = None) -> Result:
    res = Result()
    st = _load().mp_solve_omp(ctx, y_ptr, x_ptr, r_ptr, ctypes.byref(opts), ctypes.byref(res),
                              ctypes.byref(trace) if trace is not None else None, stream)
    _check(st, "mp_solve_omp", ctx)
    return res


def mp_create_f64(psi_ptr: int, n: int, m: int, ld: int, flags: int = 0,
                  stream: Optional[int] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = _load().mp_create_f64(ctypes.byref(h), psi_ptr, n, m, ld, flags, stream)
    _check(st, "mp_create_f64", None)
    return h


def mp_create_signs(signs_ptr: int, n: int, m: int, ldw: int, flags: int = 0,
                    stream: Optional[int] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = _load().mp_create_signs(ctypes.byref(h), signs_ptr, n, m, ldw, flags, stream)
    _check(st, "mp_create_signs", None)
    return h


def mp_solve_f64(ctx, y_ptr: int, x_ptr: int, r_ptr: Optional[int], opts: Opts,
                 trace: Optional[TraceF64] = None, stream: Optional[int] = None) -> Result:
    res = Result()
    st = _load().mp_solve_f64(ctx, y_ptr, x_ptr, r_ptr, ctypes.byref(opts), ctypes.byref(res),
                              ctypes.byref(trace) if trace is not None else None, stream)
    _check(st, "mp_solve_f64", ctx)
    return res


def mp_solve_batched(ctx, y_ptr: int, ldy: int, nb: int, x_ptr: int, ldx: int,
                     r_ptr: Optional[int], ldr: int, opts: Opts, max_iters_b=None,
                     trace: Optional[Trace] = None, stream: Optional[int] = None):
    """Returns a ctypes array of ``nb`` Result structures."""
    res = (Result * max(nb, 1))()
    caps = None
    if max_iters_b is not None:
        caps = (ctypes.c_int64 * max(nb, 1))(*[int(v) for v in max_iters_b])
    st = _load().mp_solve_batched(ctx, y_ptr, ldy, nb, x_ptr, ldx, r_ptr, ldr, ctypes.byref(opts),
                                  caps, res, ctypes.byref(trace) if trace is not None else None,
                                  stream)
    _check(st, "mp_solve_batched", ctx)
    return res


def mp_create_ragged(instances, storage: int = MP_F32, flags: int = 0,
                     stream: Optional[int] = None) -> ctypes.c_void_p:
    """``instances``: sequence of (psi_ptr, n, m, ld)."""
    arr = (Instance * len(instances))(*[Instance(*t) for t in instances])
    h = ctypes.c_void_p()
    st = _load().mp_create_ragged(ctypes.byref(h), arr, len(instances), storage, flags, stream)
    _check(st, "mp_create_ragged", None)
    return h


def mp_solve_ragged(ctx, y_ptr: int, x_ptr: int, r_ptr: Optional[int], opts: Opts, count: int,
                    max_iters=None, trace: Optional[Trace] = None,
                    stream: Optional[int] = None):
    res = (Result * count)()
    caps = None
    if max_iters is not None:
        caps = (ctypes.c_int64 * count)(*[int(v) for v in max_iters])
    st = _load().mp_solve_ragged(ctx, y_ptr, x_ptr, r_ptr, ctypes.byref(opts), caps, res,
                                 ctypes.byref(trace) if trace is not None else None, stream)
    _check(st, "mp_solve_ragged", ctx)
    return res


def mp_batched_set_config(ctx, atoms128_above: int, atoms64_above: int,
                          atoms32_above: int = 0) -> None:
    cfg = BatchedConfig(atoms128_above, atoms64_above, atoms32_above)
    _check(_load().mp_batched_set_config(ctx, ctypes.byref(cfg)), "mp_batched_set_config", ctx)


def mp_batched_get_config(ctx):
    cfg = BatchedConfig()
    _check(_load().mp_batched_get_config(ctx, ctypes.byref(cfg)), "mp_batched_get_config", ctx)
    return dict(atoms128_above=cfg.atoms128_above, atoms64_above=cfg.atoms64_above,
                atoms32_above=cfg.atoms32_above)


def mp_ragged_set_config(ctx, threads: int, cols_per_wave: int, wgs_per_cu: int,
                         split: int = 0) -> None:
    cfg = RaggedConfig(threads, cols_per_wave, wgs_per_cu, split)
    _check(_load().mp_ragged_set_config(ctx, ctypes.byref(cfg)), "mp_ragged_set_config", ctx)


def mp_ragged_get_config(ctx):
    cfg = RaggedConfig()
    _check(_load().mp_ragged_get_config(ctx, ctypes.byref(cfg)), "mp_ragged_get_config", ctx)
    return dict(threads=cfg.threads, cols_per_wave=cfg.cols_per_wave, wgs_per_cu=cfg.wgs_per_cu,
                split=cfg.split)


def mp_destroy(ctx) -> None:
    _load().mp_destroy(ctx)


def mp_status_str(s: int) -> str:
    return _status_str(s)


def mp_last_error(ctx=None) -> str:
    return _load().mp_last_error(ctx).decode(errors="replace")


def mp_get_storage(ctx, codes_ptr: int, scales_ptr: Optional[int], stream=None) -> None:
    _check(_load().mp_get_storage(ctx, codes_ptr, scales_ptr, stream), "mp_get_storage", ctx)


def mp_set_profiling(ctx, every: int) -> None:
    _check(_load().mp_set_profiling(ctx, int(every)), "mp_set_profiling", ctx)


def mp_kernel_time(ctx):
    avg = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_load().mp_kernel_time(ctx, ctypes.byref(avg), ctypes.byref(n)), "mp_kernel_time",
           ctx)
    return avg.value, n.value


# ---- torch-facing convenience ------------------------------------------------

def _check_psi(psi: torch.Tensor, dtype=torch.float32):
    if not psi.is_cuda or psi.dtype != dtype or psi.dim() != 2:
        raise ValueError(f"psi must be a 2-D {dtype} CUDA tensor of shape (N, M)")
    n, m = psi.shape
    if psi.stride(0) != 1 and n > 1:
        raise ValueError("psi must be column-major: stride(0) == 1")
    ld = psi.stride(1) if m > 1 else n
    return n, m, max(ld, n)


class Decoder:
    """A dictionary prepared on the GPU (``mp_create`` / ``mp_create_f64``) and
    decodes against it.

    ``psi``: (N, M) CUDA tensor, column-major (``stride(0) == 1``): float32
    for ``storage`` ``"f32"``, ``"bf16"`` or ``"fp8"``; float64 for ``"f64"``
    (the FP64 decode: y, x~ and r are then float64 as well).  For ``"sign"``
    (``mp_create_signs``, the Bernoulli dictionary of eq. 13 as sign bits)
    ``psi`` is the packed bits, an (M, ldw) int32 CUDA tensor with contiguous
    rows, and ``n`` gives N.
    """

    def __init__(self, psi: torch.Tensor, storage: str = "f32", check_norms: bool = True,
                 stream=None, n: Optional[int] = None):
        if storage not in DTYPES:
            raise ValueError(f"unknown storage {storage!r}")
        self.dtype = torch.float64 if storage == "f64" else torch.float32
        flags = 0 if check_norms else MP_SKIP_NORM_CHECK
        if storage == "sign":
            if not psi.is_cuda or psi.dtype != torch.int32 or psi.dim() != 2 or psi.stride(1) != 1:
                raise ValueError("sign bits must be an (M, ldw) int32 CUDA tensor, rows contiguous")
            if n is None:
                raise ValueError("storage 'sign' needs n")
            m, ldw = psi.shape
            self.n, self.m, self.storage = int(n), m, storage
            ldw = psi.stride(0) if m > 1 else ldw
            self._ctx = mp_create_signs(psi.data_ptr(), int(n), m, ldw, flags,
                                        _stream_ptr(stream))
            return
        n, m, ld = _check_psi(psi, self.dtype)
        self.n, self.m, self.storage = n, m, storage
        if storage == "f64":
            self._ctx = mp_create_f64(psi.data_ptr(), n, m, ld, flags, _stream_ptr(stream))
        else:
            self._ctx = mp_create(psi.data_ptr(), n, m, ld, DTYPES[storage], flags,
                                  _stream_ptr(stream))

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            mp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._ctx

    def solve(self, y: torch.Tensor, eps: float, max_iters: int, x: Optional[torch.Tensor] = None,
              r: Optional[torch.Tensor] = None, trace_cap: int = 0, rescore_k: int = 0,
              stream=None, omp: bool = False, step_launches: bool = False,
              trace_r: bool = False, noalloc: bool = False, asynchronous: bool = False):
        """Decode one signal.  Returns dict(x, r, iters, yy, rr, stop, persistent,
        trace...).  ``omp=True`` decodes with Orthogonal Matching Pursuit
        (mp_solve_omp; MP_F32 storage).  ``step_launches=True``: the one-bit
        form steps with one launch per iteration (MP_SOLVE_STEP_LAUNCHES).
        ``trace_r=True`` (with ``trace_cap``): also the residual after every
        traced step, ``r_trace`` of shape (steps, N).  ``noalloc=True``:
        mp_solve_noalloc (the library's static scratch; MP_F32, MP_BF16 or
        MP_FP8_E4M3 storage).  ``asynchronous=True``: a stream-ordered decode
        (MP_SOLVE_ASYNC): returns dict(x, r, and the whole trace arrays) at
        once, final when ``stream`` gets there; ``result()`` then waits and
        gives the rest."""
        dt = self.dtype
        if not y.is_cuda or y.dtype != dt or y.numel() != self.n:
            raise ValueError(f"y must be a {dt} CUDA tensor of N elements")
        y = y.contiguous()
        dev = y.device
        if x is None:
            x = torch.empty(self.m, dtype=dt, device=dev)
        if r is None:
            r = torch.empty(self.n, dtype=dt, device=dev)
        tr = None
        tidx = tcoef = trr = tres = None
        if trace_cap > 0:
            tidx = torch.full((trace_cap,), -1, dtype=torch.int32, device=dev)
            tcoef = torch.zeros(trace_cap, dtype=dt, device=dev)
            trr = torch.zeros(trace_cap, dtype=torch.float64, device=dev)
            if trace_r:
                tres = torch.zeros((trace_cap, self.n), dtype=dt, device=dev)
            tr = (TraceF64 if self.storage == "f64" else Trace)(
                tidx.data_ptr(), tcoef.data_ptr(), trr.data_ptr(), trace_cap, _ptr(tres), self.n)
        opts = Opts(float(eps), int(max_iters), int(rescore_k),
                    (MP_SOLVE_STEP_LAUNCHES if step_launches else 0) |
                    (MP_SOLVE_ASYNC if asynchronous else 0))
        if omp and self.storage != "f32":
            raise ValueError("OMP decodes need f32 storage")
        if noalloc and (omp or self.storage in ("f64", "sign")):
            raise ValueError("noalloc decodes need f32, bf16 or fp8 storage and plain MP")
        if asynchronous:
            if omp or self.storage in ("f64", "sign"):
                raise ValueError("stream-ordered decodes need f32, bf16 or fp8 storage and "
                                 "plain MP")
            solve = mp_solve_noalloc if noalloc else mp_solve
            solve(self._ctx, y.data_ptr(), x.data_ptr(), r.data_ptr(), opts, tr,
                  _stream_ptr(stream), want_result=False)
            out = dict(x=x, r=r)
            if tr is not None:
                out.update(idx=tidx, coef=tcoef, rr_trace=trr)
                if tres is not None:
                    out.update(r_trace=tres)
            return out
        solve = mp_solve_f64 if self.storage == "f64" else (
            mp_solve_omp if omp else (mp_solve_noalloc if noalloc else mp_solve))
        res = solve(self._ctx, y.data_ptr(), x.data_ptr(), r.data_ptr(), opts, tr,
                    _stream_ptr(stream))
        out = dict(x=x, r=r, iters=res.iters, yy=res.yy, rr=res.rr,
                   stop=STOP_NAMES.get(res.stop_reason, res.stop_reason),
                   persistent=bool(res.persistent))
        if tr is not None:
            k = min(res.iters, trace_cap)
            out.update(idx=tidx[:k], coef=tcoef[:k], rr_trace=trr[:k])
            if tres is not None:
                out.update(r_trace=tres[:k])
        return out

    def result(self):
        """Wait for the stream-ordered decode last issued on this decoder and
        return dict(iters, yy, rr, stop, persistent) (mp_solve_result)."""
        res = mp_solve_result(self._ctx)
        return dict(iters=res.iters, yy=res.yy, rr=res.rr,
                    stop=STOP_NAMES.get(res.stop_reason, res.stop_reason),
                    persistent=bool(res.persistent))

    def set_batched_config(self, atoms128_above: int, atoms64_above: int,
                           atoms32_above: int = 0) -> None:
        """Product tile rule of solve_batched: 128 atoms while more than
        atoms128_above signals are active, 64 while more than atoms64_above,
        32 while more than atoms32_above, else 16."""
        mp_batched_set_config(self._ctx, atoms128_above, atoms64_above, atoms32_above)

    def get_batched_config(self):
        return mp_batched_get_config(self._ctx)

    def solve_batched(self, y: torch.Tensor, eps: float, max_iters, trace_cap: int = 0,
                      rescore_k: int = 0, want_r: bool = True, stream=None,
                      trace_r: bool = False):
        """Decode the columns of ``y`` ((N, B) float32 CUDA, column-major).

        ``max_iters``: one cap for all signals, or a sequence of B caps.
        Returns dict(x (M, B), r (N, B) or None, iters, yy, rr, stop (lists), and
        with ``trace_cap`` idx/coef/rr_trace of shape (B, trace_cap); with
        ``trace_r`` also r_trace of shape (B, trace_cap, N))."""
        if not y.is_cuda or y.dtype != torch.float32 or y.dim() != 2 or y.shape[0] != self.n:
            raise ValueError("y must be a (N, B) float32 CUDA tensor")
        nb = y.shape[1]
        if nb > 1 and y.stride(0) != 1:
            raise ValueError("y must be column-major: stride(0) == 1")
        ldy = max(y.stride(1) if nb > 1 else self.n, self.n)
        dev = y.device
        x = torch.empty((max(nb, 1), self.m), dtype=torch.float32, device=dev)
        r = torch.empty((max(nb, 1), self.n), dtype=torch.float32, device=dev) if want_r else None
        tr = None
        tidx = tcoef = trr = tres = None
        if trace_cap > 0:
            tidx = torch.full((max(nb, 1), trace_cap), -1, dtype=torch.int32, device=dev)
            tcoef = torch.zeros((max(nb, 1), trace_cap), dtype=torch.float32, device=dev)
            trr = torch.zeros((max(nb, 1), trace_cap), dtype=torch.float64, device=dev)
            if trace_r:
                tres = torch.zeros((max(nb, 1), trace_cap, self.n), dtype=torch.float32,
                                   device=dev)
            tr = Trace(tidx.data_ptr(), tcoef.data_ptr(), trr.data_ptr(), trace_cap, _ptr(tres),
                       self.n)
        per = None
        if isinstance(max_iters, (list, tuple)) or hasattr(max_iters, "__len__"):
            per = [int(v) for v in max_iters]
            if len(per) != nb:
                raise ValueError("need one cap per signal")
            cap_all = max(per) if per else 0
        else:
            cap_all = int(max_iters)
        opts = Opts(float(eps), cap_all, int(rescore_k), 0)
        res = mp_solve_batched(self._ctx, y.data_ptr(), ldy, nb, x.data_ptr(), self.m,
                               _ptr(r), self.n, opts, per, tr, _stream_ptr(stream))
        out = dict(x=x[:nb].t(), r=None if r is None else r[:nb].t(),
                   iters=[res[i].iters for i in range(nb)], yy=[res[i].yy for i in range(nb)],
                   rr=[res[i].rr for i in range(nb)],
                   stop=[STOP_NAMES.get(res[i].stop_reason, res[i].stop_reason)
                         for i in range(nb)])
        if tr is not None:
            out.update(idx=tidx[:nb], coef=tcoef[:nb], rr_trace=trr[:nb])
            if tres is not None:
                out.update(r_trace=tres[:nb])
        return out

    def storage_copy(self, stream=None):
        """The dictionary copy the correlation pass streams, unpadded:
        (codes tensor (N, M) column-major view, scales or None); for "sign"
        storage the packed bits, (M, ceil(N/32)) int32, and None."""
        if self.storage == "sign":
            codes = torch.empty((self.m, (self.n + 31) // 32), dtype=torch.int32, device="cuda")
            mp_get_storage(self._ctx, codes.data_ptr(), None, _stream_ptr(stream))
            return codes, None
        dt = {"f32": torch.float32, "bf16": torch.int16, "fp8": torch.uint8,
              "f64": torch.float64}[self.storage]
        codes = torch.empty((self.m, self.n), dtype=dt, device="cuda")
        scales = torch.empty(self.m, dtype=torch.float32, device="cuda") \
            if self.storage == "fp8" else None
        mp_get_storage(self._ctx, codes.data_ptr(), _ptr(scales), _stream_ptr(stream))
        return codes.t(), scales

    def set_profiling(self, every: int = 1):
        """Time the step kernel's launches with HIP events (0 = off): windows of
        ``every`` consecutive launches (at most 64), OMP every ``every``-th
        selection launch on its own."""
        mp_set_profiling(self._ctx, int(every))

    def kernel_time(self):
        """(mean correlation-kernel launch time in ms, launches counted)."""
        return mp_kernel_time(self._ctx)


class RaggedDecoder:
    """Independent problems of uneven size (``mp_create_ragged``).

    ``psis``: list of (N_i, M_i) float32 CUDA tensors, column-major.
    """

    def __init__(self, psis, storage: str = "f32", check_norms: bool = True, stream=None):
        descs = []
        self.ns, self.ms = [], []
        for psi in psis:
            n, m, ld = _check_psi(psi)
            descs.append((psi.data_ptr(), n, m, ld))
            self.ns.append(n)
            self.ms.append(m)
        self.count = len(descs)
        self.storage = storage
        flags = 0 if check_norms else MP_SKIP_NORM_CHECK
        self._ctx = mp_create_ragged(descs, DTYPES[storage], flags, _stream_ptr(stream))
        self.y_off = [0]
        self.x_off = [0]
        for n, m in zip(self.ns, self.ms):
            self.y_off.append(self.y_off[-1] + n)
            self.x_off.append(self.x_off[-1] + m)

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            mp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._ctx

    def set_config(self, threads: int, cols_per_wave: int, wgs_per_cu: int, split: int = 0):
        """Launch shape; ``split``: most parts one instance is cut into (0:
        the library's default)."""
        mp_ragged_set_config(self._ctx, threads, cols_per_wave, wgs_per_cu, split)

    def get_config(self):
        return mp_ragged_get_config(self._ctx)

    def pack(self, ys):
        """Concatenate per-instance y tensors into the packed layout."""
        return torch.cat([y.reshape(-1) for y in ys]).contiguous()

    def solve(self, y_packed: torch.Tensor, eps: float, max_iters, trace_cap: int = 0,
              rescore_k: int = 0, want_r: bool = True, x_out=None, stream=None,
              trace_r: bool = False):
        """Decode every instance.  ``y_packed``: float32 CUDA vector of sum(N_i).
        ``max_iters``: one cap, or one per instance.  Returns dict with packed
        ``x``/``r`` and per-instance ``iters``/``stop``/``yy``/``rr`` lists,
        plus ``idx``/``coef``/``rr_trace`` (count, trace_cap) with a trace and,
        with ``trace_r``, ``r_trace`` (count, trace_cap, max N_i): instance i's
        residual after step t in the first N_i entries of [i, t]."""
        if (not y_packed.is_cuda or y_packed.dtype != torch.float32
                or y_packed.numel() != self.y_off[-1]):
            raise ValueError("y_packed must be a float32 CUDA vector of sum(N_i) entries")
        y_packed = y_packed.contiguous()
        dev = y_packed.device
        x = x_out if x_out is not None else torch.empty(self.x_off[-1], dtype=torch.float32,
                                                         device=dev)
        r = torch.empty(self.y_off[-1], dtype=torch.float32, device=dev) if want_r else None
        tr = None
        tidx = tcoef = trr = tres = None
        if trace_cap > 0:
            tidx = torch.full((self.count, trace_cap), -1, dtype=torch.int32, device=dev)
            tcoef = torch.zeros((self.count, trace_cap), dtype=torch.float32, device=dev)
            trr = torch.zeros((self.count, trace_cap), dtype=torch.float64, device=dev)
            ldr = max(self.ns)
            if trace_r:
                tres = torch.zeros((self.count, trace_cap, ldr), dtype=torch.float32, device=dev)
            tr = Trace(tidx.data_ptr(), tcoef.data_ptr(), trr.data_ptr(), trace_cap, _ptr(tres),
                       ldr)
        per = None
        if hasattr(max_iters, "__len__"):
            per = [int(v) for v in max_iters]
            if len(per) != self.count:
                raise ValueError("need one cap per instance")
            cap_all = max(per)
        else:
            cap_all = int(max_iters)
        opts = Opts(float(eps), cap_all, int(rescore_k), 0)
        res = mp_solve_ragged(self._ctx, y_packed.data_ptr(), x.data_ptr(), _ptr(r), opts,
                              self.count, per, tr, _stream_ptr(stream))
        out = dict(x=x, r=r, iters=[res[i].iters for i in range(self.count)],
                   yy=[res[i].yy for i in range(self.count)],
                   rr=[res[i].rr for i in range(self.count)],
                   stop=[STOP_NAMES.get(res[i].stop_reason, res[i].stop_reason)
                         for i in range(self.count)])
        if tr is not None:
            out.update(idx=tidx, coef=tcoef, rr_trace=trr)
            if tres is not None:
                out.update(r_trace=tres)
        return out

    def set_profiling(self, every: int = 1):
        mp_set_profiling(self._ctx, int(every))

    def kernel_time(self):
        return mp_kernel_time(self._ctx)
