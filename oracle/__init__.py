"""CPU oracle for the Matching Pursuit decoder.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import anything from this package.
The GPU library never calls it and shares no code with it.

Contents
* :func:`solve` / :func:`solve64` / :func:`correlate` -- the plain FP64 MP of
  Section 3 (eqs. 8-12, argmax tie rule of eq. 16), in C (``mp_oracle.c``);
  ``solve`` takes y as FP32 (the FP32 decoder's input), ``solve64`` an FP64
  dictionary and an FP64 y (the FP64 decoder's inputs).
* :func:`replay` -- the same FP64 iteration following a given index sequence
  instead of eq. 9's selection (C), optionally with each forced atom's deficit
  against the FP64 maximum.
* :func:`correlate_many` / :class:`Correlator` / :func:`top_gap` -- eq. 9's
  correlations of many vectors at once (an FP64 matrix product), and per
  vector the smallest-index argmax and the top-two gap.
* :mod:`oracle.omp` -- Orthogonal Matching Pursuit in FP64 (MP's selection,
  least-squares re-fit of all selected atoms).
* :mod:`oracle.signs` -- the Bernoulli dictionary of eq. 13 held as sign bits,
  read back into FP64 entries +-1/sqrt(N) and decoded by the FP64 MP above.
* :mod:`oracle.exact` -- exact rational MP and OMP, brute-force pins.
* :mod:`oracle.quant` -- reference BF16 / FP8-e4m3fn quantisers.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmporacle.so")

CONVERGED, MAX_ITERS, STALLED, ZERO_INPUT = 0, 1, 2, 3
REASONS = {CONVERGED: "converged", MAX_ITERS: "max_iters", STALLED: "stalled",
           ZERO_INPUT: "zero_input"}

_lib = None


def load_library(path: str):
    """Open a compiled oracle (the default one, or a test-built variant)."""
    lib = ctypes.CDLL(path)
    p, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    for name in ("f32", "f64", "f64_y64"):
        f = getattr(lib, "mpo_solve_" + name)
        f.restype = ctypes.c_int
        f.argtypes = [p, i64, i64, i64, p, dbl, i64, p, p, p, p, p, p, p, p, p, p, i64]
    for name in ("f32", "f64", "f64_y64"):
        f = getattr(lib, "mpo_replay_" + name)
        f.restype = ctypes.c_int
        f.argtypes = [p, i64, i64, i64, p, p, i64, ctypes.c_int, p, p, p, p, p, p]
    for suf in ("f32", "f64"):
        g = getattr(lib, "mpo_correlate_" + suf)
        g.restype = None
        g.argtypes = [p, i64, i64, i64, p, p]
    lib.mpo_num_threads.restype = ctypes.c_int
    lib.mpo_set_num_threads.argtypes = [ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    _lib = load_library(LIB_PATH)
    return _lib


def num_threads() -> int:
    return _load().mpo_num_threads()


def set_num_threads(n: int) -> None:
    _load().mpo_set_num_threads(int(n))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _psi_view(psi: np.ndarray):
    """(pointer-able array, suffix, n, m, ld) for a column-major dictionary."""
    if psi.ndim != 2:
        raise ValueError("psi must be 2-D (N, M)")
    n, m = psi.shape
    if psi.dtype == np.float32:
        suf = "f32"
    elif psi.dtype == np.float64:
        suf = "f64"
    else:
        raise TypeError("psi must be float32 or float64")
    if psi.flags.f_contiguous:
        base, ld = psi, n
    else:
        base, ld = np.asfortranarray(psi), n
    return base, suf, n, m, ld


@dataclass
class Result:
    x: np.ndarray          # (M,) float64 estimate x~
    r: np.ndarray          # (N,) float64 residual
    iters: int
    reason: int
    yy: float              # ||y||^2
    rr: float              # ||r||^2 at exit
    idx: np.ndarray        # (iters,) int32 selected indices (trace)
    coef: np.ndarray       # (iters,) float64 selected coefficients
    rr_trace: np.ndarray   # (iters,) float64 ||r||^2 after each step
    gap: np.ndarray        # (iters,) float64 top-two |c| gap before each step


def solve(psi: np.ndarray, y: np.ndarray, eps: float, max_iters: int,
          trace: bool = True, lib=None) -> Result:
    """FP64 Matching Pursuit on the given dictionary (FP32 or FP64 storage) and
    an FP32 y (y is rounded to FP32 first, as the FP32 decoder receives it)."""
    lib = _load() if lib is None else lib
    base, suf, n, m, ld = _psi_view(psi)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    if y32.shape != (n,):
        raise ValueError("y must have shape (N,)")
    return _run(lib, "mpo_solve_" + suf, base, n, m, ld, y32, eps, max_iters, trace)


def solve64(psi: np.ndarray, y: np.ndarray, eps: float, max_iters: int,
            trace: bool = True, lib=None) -> Result:
    """The same FP64 Matching Pursuit on an FP64 dictionary and an FP64 y (the
    inputs of the FP64 decoder), with no rounding of either."""
    lib = _load() if lib is None else lib
    if psi.dtype != np.float64:
        raise TypeError("solve64 needs a float64 dictionary")
    base, _, n, m, ld = _psi_view(psi)
    y64 = np.ascontiguousarray(y, dtype=np.float64)
    if y64.shape != (n,):
        raise ValueError("y must have shape (N,)")
    return _run(lib, "mpo_solve_f64_y64", base, n, m, ld, y64, eps, max_iters, trace)


def _run(lib, fname, base, n, m, ld, yv, eps, max_iters, trace):
    x = np.zeros(m, dtype=np.float64)
    r = np.zeros(n, dtype=np.float64)
    iters = np.zeros(1, dtype=np.int64)
    reason = np.zeros(1, dtype=np.int32)
    yy = np.zeros(1, dtype=np.float64)
    rr = np.zeros(1, dtype=np.float64)
    cap = int(max_iters) if trace else 0
    ti = np.zeros(max(cap, 1), dtype=np.int32)
    tc = np.zeros(max(cap, 1), dtype=np.float64)
    tr = np.zeros(max(cap, 1), dtype=np.float64)
    tg = np.zeros(max(cap, 1), dtype=np.float64)
    rc = getattr(lib, fname)(
        _ptr(base), n, m, ld, _ptr(yv), float(eps), int(max_iters),
        _ptr(x), _ptr(r), _ptr(iters), _ptr(reason), _ptr(yy), _ptr(rr),
        _ptr(ti), _ptr(tc), _ptr(tr), _ptr(tg), cap)
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (code {rc})")
    t = int(iters[0])
    k = min(t, cap)
    return Result(x, r, t, int(reason[0]), float(yy[0]), float(rr[0]),
                  ti[:k].copy(), tc[:k].copy(), tr[:k].copy(), tg[:k].copy())


def correlate(psi: np.ndarray, r: np.ndarray, lib=None) -> np.ndarray:
    """c = Psi^T r in FP64 (eq. 9's inner products), sequential per column."""
    lib = _load() if lib is None else lib
    base, suf, n, m, ld = _psi_view(psi)
    r64 = np.ascontiguousarray(r, dtype=np.float64)
    if r64.shape != (n,):
        raise ValueError("r must have shape (N,)")
    c = np.zeros(m, dtype=np.float64)
    getattr(lib, "mpo_correlate_" + suf)(_ptr(base), n, m, ld, _ptr(r64), _ptr(c))
    return c


@dataclass
class Replay:
    x: np.ndarray          # (M,) float64 estimate after the forced steps
    r: np.ndarray          # (N,) float64 residual after them
    coef: np.ndarray       # (steps,) float64 FP64 coefficient of each forced step
    rr_trace: np.ndarray   # (steps,) float64 ||r||^2 after each step
    deficit: np.ndarray    # (steps,) max |c| - |c_forced| before each step (0 unchecked)
    r_trace: Optional[np.ndarray]  # (steps, N) float64 r after each step, if asked


def replay(psi: np.ndarray, y: np.ndarray, idx, check_ties: bool = True,
           r_trace: bool = False, y64: bool = False, lib=None) -> Replay:
    """The Section 3 iteration in FP64 with step t's atom forced to idx[t]
    (eq. 9's selection replaced; eqs. 10-11 unchanged).  ``check_ties``: also
    compute every correlation at every step and record the forced atom's
    deficit max_m |c_m| - |c_idx|.  ``y64``: y is taken in FP64 (an FP64
    dictionary only), else rounded to FP32 as :func:`solve` does."""
    lib = _load() if lib is None else lib
    base, suf, n, m, ld = _psi_view(psi)
    if y64:
        if psi.dtype != np.float64:
            raise TypeError("an FP64 y needs a float64 dictionary")
        yv, fname = np.ascontiguousarray(y, dtype=np.float64), "mpo_replay_f64_y64"
    else:
        yv, fname = np.ascontiguousarray(y, dtype=np.float32), "mpo_replay_" + suf
    if yv.shape != (n,):
        raise ValueError("y must have shape (N,)")
    ix = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1)
    steps = ix.size
    x = np.zeros(m, dtype=np.float64)
    r = np.zeros(n, dtype=np.float64)
    coef = np.zeros(max(steps, 1), dtype=np.float64)
    rr = np.zeros(max(steps, 1), dtype=np.float64)
    dfc = np.zeros(max(steps, 1), dtype=np.float64)
    rt = np.zeros((steps, n), dtype=np.float64) if r_trace else None
    rc = getattr(lib, fname)(_ptr(base), n, m, ld, _ptr(yv), _ptr(ix) if steps else None, steps,
                             1 if check_ties else 0, _ptr(x), _ptr(r), _ptr(coef), _ptr(rr),
                             _ptr(dfc), _ptr(rt) if steps else None)
    if rc != 0:
        raise ValueError(f"oracle rejected the replay (code {rc})")
    return Replay(x, r, coef[:steps].copy(), rr[:steps].copy(), dfc[:steps].copy(), rt)


class Correlator:
    """Eq. 9's correlations of many vectors against one dictionary: keeps the
    dictionary's FP64 transpose (M x N, one row per atom) so that repeated
    calls do not convert it again.  ``many(R)`` is :func:`correlate_many`."""

    def __init__(self, psi: np.ndarray):
        import torch
        self.n, self.m = psi.shape
        self._P = torch.from_numpy(np.asarray(psi, dtype=np.float64).T.copy())

    def many(self, R: np.ndarray, chunk: int = 512) -> np.ndarray:
        import torch
        R = np.asarray(R)
        if R.ndim != 2 or R.shape[0] != self.n:
            raise ValueError("R must have shape (N, K)")
        out = np.empty((self.m, R.shape[1]), dtype=np.float64)
        for j0 in range(0, R.shape[1], chunk):
            j1 = min(R.shape[1], j0 + chunk)
            Rc = torch.from_numpy(np.ascontiguousarray(R[:, j0:j1], dtype=np.float64))
            out[:, j0:j1] = (self._P @ Rc).numpy()
        return out


def correlate_many(psi: np.ndarray, R: np.ndarray, chunk: int = 512) -> np.ndarray:
    """C[:, j] = Psi^T R[:, j] in FP64 for every column of R (N x K): eq. 9's
    correlations of K vectors, computed as one FP64 matrix product per chunk
    of columns (torch on the CPU).  The summation order is the library's, so
    each value differs from :func:`correlate`'s sequential sum only by FP64
    rounding."""
    return Correlator(psi).many(R, chunk=chunk)


def top_gap(C: np.ndarray):
    """Per column of C (M x K): the argmax of |c| with eq. 16's smallest-index
    rule, the largest |c| and the gap to the second largest (0 for M = 1:
    the largest |c| itself)."""
    a = np.abs(np.asarray(C, dtype=np.float64))
    best = np.argmax(a, axis=0)  # first occurrence: the smallest index
    top = a[best, np.arange(a.shape[1])]
    if a.shape[0] == 1:
        return best, top, top.copy()
    second = -np.partition(-a, 1, axis=0)[1]
    return best, top, top - second
