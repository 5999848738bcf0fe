"""Whole-run parity of a GPU decode against the FP64 oracle (test helper).

A GPU decode run with a residual trace (``mp_trace.r``) hands over its state
r_t before every step t (r_0 = y) together with its selections and
coefficients.  Three checks then cover every step of the run, however long:

P-local (Section 3, eq. 9 with the i?amax rule of eq. 16).  The oracle
correlates each GPU state in FP64 (``oracle.Correlator``).  Wherever the
top-two gap of |c| exceeds ``tol_sel * ||r_t||`` the GPU's atom must be the
FP64 argmax exactly; everywhere its |c| must be within ``tol_sel * ||r_t|| +
2 e32`` of the maximum (e32 bounds the FP32 inner-product rounding), and its
coefficient must equal the FP64 one within e32.  A selection that differs
where the gap is larger is a miss (for the reduced-precision forms: the FP32
winner was not among the re-scored candidates); misses must be 0.

P-replay (eqs. 10-11).  The oracle replays the GPU's index sequence in FP64
(``oracle.replay``).  Each forced atom must lie in the near-tie set of the
oracle's own state: max|c^o| - |c^o_i| <= tol_sel ||r^o_t|| + 2 ||r^g_t -
r^o_t|| + 2 e32.  (For unit columns |<d, psi_m>| <= ||d||, so the correlations
of the two states differ by at most ||r^g_t - r^o_t|| for every atom; the GPU
atom's deficit on its own state is at most 2 e32 plus the near-tie
allowance.)  At the end x~ and r must agree with the replay within ``tol``
(x~ relative to ||x~||, r relative to ||y||), and the replay must confirm the
stop step: above the threshold before the last step and, for a converged
run, at or below it after, up to the drift of ||r||^2.

End state.  y = Psi x~ + r for the GPU result.

Nothing the GPU returns becomes an expected value: GPU states are only
evaluated by the oracle, and every comparison is against oracle output.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

import oracle
from parity import U32, fp32_dot_bound


@dataclass
class WholeRunReport:
    steps: int
    exact_steps: int = 0          # steps whose gap demanded the exact argmax
    near_ties: int = 0            # differing selections allowed by a small gap
    misses: int = 0               # differing selections at a larger gap (must be 0)
    max_sel_slack: float = 0.0    # max over steps of (max|c| - |c_i|) / ||r_t||
    max_coef_err: float = 0.0     # max |coef - c_i| / (e32 + rel |c_i|)  (<= 1)
    max_replay_deficit: float = 0.0  # max deficit / allowed on the oracle's states (<= 1)
    max_dr: float = 0.0           # max ||r^g_t - r^o_t|| / ||y||
    x_err: float = 0.0
    r_err: float = 0.0
    notes: List[str] = field(default_factory=list)


def _stack_states(y: np.ndarray, rtrace: np.ndarray, a: int, b: int) -> np.ndarray:
    """States before steps a..b-1 as an (N, b-a) FP64 matrix: r_0 = y,
    r_t = the trace entry of step t - 1."""
    cols = []
    for t in range(a, b):
        cols.append(y if t == 0 else rtrace[t - 1])
    return np.asarray(np.stack(cols, axis=1), dtype=np.float64)


def _inputs(y, g, y64):
    T = int(g["iters"])
    idx = np.asarray(g["idx"], dtype=np.int64)[:T]
    coef = np.asarray(g["coef"], dtype=np.float64)[:T]
    rtr = np.asarray(g["r_trace"])[:T]
    assert idx.size == T and coef.size == T and rtr.shape[0] == T, "trace shorter than the run"
    yv = np.asarray(y, dtype=np.float64) if y64 else np.asarray(y, dtype=np.float32).astype(
        np.float64)
    return T, idx, coef, rtr, yv


def local_checks(psi: np.ndarray, y: np.ndarray, g: dict, tol_sel: float = 1e-5,
                 unit: float = U32, y64: bool = False, chunk: int = 1024,
                 coef_rel: Optional[float] = None, corr=None) -> WholeRunReport:
    """P-local alone (any decode whose step t selects by eq. 9 on its state
    r_t and records that atom's correlation: MP in every form, and OMP)."""
    n, m = psi.shape
    T, idx, coef, rtr, yv = _inputs(y, g, y64)
    rep = WholeRunReport(T)
    if corr is None:
        corr = oracle.Correlator(psi)
    if coef_rel is None:
        coef_rel = 1e-6 if unit == U32 else 16 * unit
    for a in range(0, T, chunk):
        b = min(T, a + chunk)
        R = _stack_states(yv, rtr, a, b)
        C = corr.many(R)
        best, top, gap = oracle.top_gap(C)
        rn = np.linalg.norm(R, axis=0)
        cols = np.arange(b - a)
        ci = C[idx[a:b], cols]
        e32 = fp32_dot_bound(n, rn, unit)
        exact = gap > tol_sel * rn
        differ = idx[a:b] != best
        rep.exact_steps += int(exact.sum())
        rep.misses += int((differ & exact).sum())
        rep.near_ties += int((differ & ~exact).sum())
        slack = (top - np.abs(ci)) / np.maximum(rn, 1e-300)
        rep.max_sel_slack = max(rep.max_sel_slack, float(slack.max(initial=0.0)))
        ok_sel = np.abs(ci) >= top - (tol_sel * rn + 2 * e32)
        bad = np.flatnonzero(~ok_sel)
        assert bad.size == 0, (f"step {a + bad[0]}: atom {idx[a + bad[0]]} |c|={abs(ci[bad[0]]):.6g}"
                               f" vs max {top[bad[0]]:.6g}")
        cerr = np.abs(coef[a:b] - ci) / (e32 + coef_rel * np.abs(ci))
        rep.max_coef_err = max(rep.max_coef_err, float(cerr.max(initial=0.0)))
        bad = np.flatnonzero(cerr > 1.0)
        assert bad.size == 0, (f"step {a + bad[0]}: coefficient {coef[a + bad[0]]!r} vs FP64 "
                               f"{ci[bad[0]]!r}")
        del C, R
    assert rep.misses == 0, f"{rep.misses} selections differ from the FP64 argmax at a gap > tol"
    return rep


def whole_run(psi: np.ndarray, y: np.ndarray, eps: float, g: dict, tol: float = 1e-5,
              tol_sel: float = 1e-5, unit: float = U32, y64: bool = False,
              oracle_ties: bool = True, chunk: int = 1024,
              coef_rel: Optional[float] = None, corr=None) -> WholeRunReport:
    """``g``: the GPU decode as numpy arrays: x, r, iters, stop, idx, coef,
    r_trace (steps x N, the residual after each step).  ``y64``: y is FP64
    (the FP64 decode); otherwise the oracle takes y rounded to FP32.
    ``oracle_ties``: also correlate the replay's states (the literal near-tie
    check on the oracle side; costs a second FP64 product).  ``corr``: an
    ``oracle.Correlator`` of psi to reuse across calls."""
    n, m = psi.shape
    if corr is None:
        corr = oracle.Correlator(psi)
    rep = local_checks(psi, y, g, tol_sel=tol_sel, unit=unit, y64=y64, chunk=chunk,
                       coef_rel=coef_rel, corr=corr)
    T, idx, coef, rtr, yv = _inputs(y, g, y64)
    ynorm = float(np.linalg.norm(yv))

    # ---- P-replay: the oracle follows the GPU's atoms ------------------------
    ora = oracle.replay(psi, yv if y64 else np.asarray(y, dtype=np.float32), idx.astype(np.int32),
                        check_ties=False, r_trace=True, y64=y64)
    ort = ora.r_trace  # (T, N): oracle residual after each step
    drs = np.zeros(T)
    for a in range(0, T, chunk):
        b = min(T, a + chunk)
        Rg = _stack_states(yv, rtr, a, b)
        Ro = _stack_states(yv, ort, a, b)
        dr = np.linalg.norm(Rg - Ro, axis=0)
        drs[a:b] = dr
        if oracle_ties:
            C = corr.many(Ro)
            _, top, _ = oracle.top_gap(C)
            ci = np.abs(C[idx[a:b], np.arange(b - a)])
            rno = np.linalg.norm(Ro, axis=0)
            allowed = tol_sel * rno + 2 * dr + 2 * fp32_dot_bound(n, rno, unit)
            ratio = (top - ci) / np.maximum(allowed, 1e-300)
            rep.max_replay_deficit = max(rep.max_replay_deficit, float(ratio.max(initial=0.0)))
            bad = np.flatnonzero(ratio > 1.0)
            assert bad.size == 0, (f"step {a + bad[0]}: forced atom {idx[a + bad[0]]} is "
                                   f"{top[bad[0]] - ci[bad[0]]:.3g} below the oracle's maximum")
            del C
    rep.max_dr = float(drs.max(initial=0.0)) / max(ynorm, 1e-300)
    if T:
        xo = ora.x
        rep.x_err = float(np.linalg.norm(np.asarray(g["x"], np.float64) - xo)) / max(
            float(np.linalg.norm(xo)), 1e-300)
        rep.r_err = float(np.linalg.norm(np.asarray(g["r"], np.float64) - ora.r)) / max(
            ynorm, 1e-300)
        assert rep.x_err <= tol, f"x~ error {rep.x_err:.3g} against the replay"
        assert rep.r_err <= tol, f"r error {rep.r_err:.3g} against the replay"

    # the replay confirms the stop step, up to the drift of ||r||^2
    thr = eps * eps * ynorm ** 2
    if T:
        dr_end = float(np.linalg.norm(np.asarray(g["r"], np.float64) - ora.r))
        rr_end = float(ora.rr_trace[-1])
        slack_end = 2.0 * np.sqrt(max(rr_end, thr)) * dr_end + dr_end ** 2
        if g["stop"] == "converged":
            assert rr_end <= thr * (1 + 1e-6) + 1.01 * slack_end, (rr_end, thr)
        rr_prev = float(ora.rr_trace[-2]) if T >= 2 else ynorm ** 2
        dr_prev = drs[T - 1]
        slack_prev = 2.0 * np.sqrt(max(rr_prev, thr)) * dr_prev + dr_prev ** 2
        assert rr_prev > thr * (1 - 1e-6) - 1.01 * slack_prev, (
            f"the oracle state before the last step is already below the threshold "
            f"({rr_prev:.6g} <= {thr:.6g})")

    # ---- end state: y = Psi x~ + r ------------------------------------------
    defect = yv - np.asarray(psi, dtype=np.float64) @ np.asarray(g["x"], np.float64) - np.asarray(
        g["r"], np.float64)
    assert np.linalg.norm(defect) <= max(tol, 4 * unit * np.sqrt(max(T, 1))) * max(
        ynorm, 1e-300) + 1e-30, "y != Psi x~ + r"
    return rep
