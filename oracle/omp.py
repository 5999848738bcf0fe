"""Orthogonal Matching Pursuit in FP64: the refinement of MP that the paper
names as the next algorithm to port (its conclusion).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The selection is MP's (eq. 9 with the smallest-index tie rule of eq. 16);
after every selection the coefficients of all selected atoms are fitted again
by least squares, so the residual is orthogonal to every selected atom.  The
paper does not spell OMP out; this is the standard definition, written out
directly:

    S = (), r = y, t = 0
    while ||r||^2 > eps^2 ||y||^2 and t < T:
        c   = Psi^T r                         (FP64 inner products)
        i   = smallest index of max_m |c_m|
        stop (STALLED) if c_i == 0 or i is already in S
        S   = S + (i)
        x_S = argmin_z ||y - Psi_S z||_2      (LAPACK least squares, FP64)
        r   = y - Psi_S x_S
        t  += 1

The per-step record holds the selected index, its correlation c_i, ||r||^2
after the step and the top-two |c| gap.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import correlate

CONVERGED, MAX_ITERS, STALLED, ZERO_INPUT = 0, 1, 2, 3
REASONS = {CONVERGED: "converged", MAX_ITERS: "max_iters", STALLED: "stalled",
           ZERO_INPUT: "zero_input"}


@dataclass
class OmpResult:
    x: np.ndarray          # (M,) float64 estimate x~
    r: np.ndarray          # (N,) float64 residual
    iters: int
    reason: int
    yy: float
    rr: float
    idx: np.ndarray        # (iters,) selected indices in order
    coef: np.ndarray       # (iters,) correlation c_i of each selected atom
    rr_trace: np.ndarray   # (iters,) ||r||^2 after each step
    gap: np.ndarray        # (iters,) top-two |c| gap before each step


# the steps as module-level helpers (the tests plant mistakes in them)
def _argmax_abs(c: np.ndarray):
    a = np.abs(c)
    i = int(np.argmax(a))  # first occurrence: the smallest index of the maximum
    second = float(np.max(np.delete(a, i))) if a.size > 1 else 0.0
    return i, float(a[i]) - second


def _fit(psi_s: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.linalg.lstsq(psi_s, y, rcond=None)[0]


def _residual(y: np.ndarray, psi_s: np.ndarray, xs: np.ndarray) -> np.ndarray:
    return y - psi_s @ xs


def solve_omp(psi: np.ndarray, y: np.ndarray, eps: float, max_iters: int,
              y_dtype=np.float32) -> OmpResult:
    """OMP on ``psi`` (FP32 or FP64, used as given) and ``y`` rounded to
    ``y_dtype`` first (FP32, the FP32 decoder's input, by default)."""
    psi64 = np.asarray(psi, dtype=np.float64)
    n, m = psi64.shape
    yv = np.asarray(np.asarray(y, dtype=y_dtype), dtype=np.float64)
    r = yv.copy()
    yy = float(yv @ yv)
    thr = eps * eps * yy
    sel, coefs, rrs, gaps = [], [], [], []
    xs = np.zeros(0)
    rr = yy
    t = 0
    if yy == 0.0:
        reason = ZERO_INPUT
    else:
        while True:
            if not rr > thr:
                reason = CONVERGED
                break
            if t >= max_iters:
                reason = MAX_ITERS
                break
            c = correlate(psi, r)
            i, gap = _argmax_abs(c)
            if c[i] == 0.0 or i in sel:
                reason = STALLED
                break
            sel.append(i)
            ps = psi64[:, sel]
            xs = _fit(ps, yv)
            r = _residual(yv, ps, xs)
            rr = float(r @ r)
            coefs.append(float(c[i]))
            rrs.append(rr)
            gaps.append(gap)
            t += 1
    x = np.zeros(m)
    if sel:
        x[np.asarray(sel)] = xs
    return OmpResult(x, r, t, reason, yy, rr, np.asarray(sel, dtype=np.int32),
                     np.asarray(coefs), np.asarray(rrs), np.asarray(gaps))
