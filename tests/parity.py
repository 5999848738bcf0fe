"""Parity protocol between the GPU decoder and the FP64 oracle (test helper).

A free-running FP32 decode and the FP64 oracle start from the same seeded
inputs.  Their index sequences agree step for step until either a near tie
(several atoms are correct choices) or the FP32 rounding drift of the residual
makes the two states pick different atoms.  The checks:

1. Prefix: indices identical up to the first difference t*; at t* the GPU
   state (x~, r after t* steps, obtained by a deterministic re-run capped at
   t*) matches the oracle's within the FP32 tolerance (x~ relative to ||x~||,
   r relative to ||y||).
2. Legitimacy of a difference: at t* the oracle's top-two gap must be small
   enough that the two states may order the top atoms differently:
   gap <= tol_sel * ||r|| + 2 ||r_gpu - r_ora|| + 2 e32, where e32 bounds the
   FP32 inner-product rounding error.
3. Validity after it: at sampled later steps s the GPU's own state r_s is
   correlated in FP64 (by the oracle) and the GPU's selected atom must be an
   argmax within tol_sel * ||r_s|| + 2 e32, with its coefficient equal to the
   FP64 one within e32.  This is a check of the GPU output; no GPU value feeds
   an expected value.
4. End state: both runs stop for the same reason (when the prefix is the
   whole run), the GPU's final residual meets the stopping rule, and
   y = Psi x~ + r holds for the GPU result to the FP32 drift tolerance.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np

import oracle

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def fp32_dot_bound(n: int, rnorm: float, unit: float = U32) -> float:
    """Bound on |fl(<r, psi>) - <r, psi>| for a unit column in the working
    precision with unit roundoff ``unit``: a lane-sequential sum of about N/64
    terms followed by a 6-level lane sum, plus FMA rounding."""
    return (n / 64.0 + 8.0) * unit * rnorm * 1.001


@dataclass
class ParityReport:
    iters_gpu: int
    iters_ora: int
    prefix: int                      # number of leading steps with identical indices
    full_match: bool
    x_err: float = 0.0               # at the prefix
    r_err: float = 0.0
    diverged_legit: bool = True
    checked_after: List[int] = field(default_factory=list)
    notes: List[str] = field(default_factory=list)


def run_parity(psi: np.ndarray, y: np.ndarray, eps: float, max_iters: int,
               gpu_solve: Callable, tol: float = 1e-5, tol_sel: float = 1e-5,
               samples_after: int = 4, oracle_cap=None, ora=None, unit: float = U32,
               solver=None) -> ParityReport:
    """``gpu_solve(eps, max_iters, trace_cap)`` -> dict of numpy arrays with keys
    x, r, iters, stop, idx, coef, rr_trace (the GPU decoder on psi, y).

    ``oracle_cap``: run the oracle for at most that many steps (large sizes);
    the prefix comparison then covers those steps and the validity checks
    sample the rest of the GPU run.  ``unit``: unit roundoff of the GPU's
    working precision (FP32 by default, ``U64`` for the FP64 decode);
    ``solver``: the oracle entry for these inputs (``oracle.solve`` by
    default, ``oracle.solve64`` for FP64 y)."""
    solver = oracle.solve if solver is None else solver
    n = psi.shape[0]
    ynorm = float(np.linalg.norm(y.astype(np.float64)))
    cap = max_iters if oracle_cap is None else min(max_iters, int(oracle_cap))
    if ora is None:
        ora = solver(psi, y, eps, cap)
    capped = cap < max_iters and ora.iters == cap
    g = gpu_solve(eps, max_iters, max_iters)
    L = min(len(g["idx"]), len(ora.idx))
    diff = np.flatnonzero(np.asarray(g["idx"][:L]) != ora.idx[:L])
    t_star = int(diff[0]) if diff.size else L
    full = t_star == L and g["iters"] == ora.iters and not capped
    rep = ParityReport(g["iters"], ora.iters, t_star, full)

    # 1. state at the end of the common prefix
    if full:
        gx, gr, ox, orr = g["x"], g["r"], ora.x, ora.r
        assert oracle.REASONS[ora.reason] == g["stop"], (ora.reason, g["stop"])
    else:
        gp = gpu_solve(0.0, t_star, 0)
        op = solver(psi, y, 0.0, t_star, trace=False)
        gx, gr, ox, orr = gp["x"], gp["r"], op.x, op.r
    xn = max(float(np.linalg.norm(ox)), 1e-300)
    rep.x_err = float(np.linalg.norm(gx.astype(np.float64) - ox)) / xn
    rep.r_err = float(np.linalg.norm(gr.astype(np.float64) - orr)) / max(ynorm, 1e-300)
    assert rep.x_err <= tol, f"x~ error {rep.x_err:.3g} at step {t_star}"
    assert rep.r_err <= tol, f"r error {rep.r_err:.3g} at step {t_star}"

    if not full:
        # 2. the first difference must be one a correct FP32 run may make
        if capped and t_star == L:
            rep.notes.append(f"oracle capped at {cap} steps; all matched")
        elif t_star < L:
            dr = float(np.linalg.norm(gr.astype(np.float64) - orr))
            rn = float(np.linalg.norm(orr))
            allowed = tol_sel * rn + 2.0 * dr + 2.0 * fp32_dot_bound(n, rn, unit)
            gap = float(ora.gap[t_star])
            rep.diverged_legit = gap <= allowed
            assert rep.diverged_legit, (
                f"step {t_star}: oracle gap {gap:.3g} exceeds allowed {allowed:.3g}")
        else:
            # one run stopped earlier: it must be at the stopping threshold
            rep.notes.append(f"stop step differs: gpu {g['iters']} oracle {ora.iters}")
        # 3. validity of the GPU's own later choices
        later = np.unique(np.linspace(t_star, max(t_star, g["iters"] - 1),
                                      num=samples_after).astype(int))
        for s in later:
            if s >= g["iters"]:
                continue
            gs = gpu_solve(0.0, int(s), 0)
            r_s = gs["r"].astype(np.float64)
            c = oracle.correlate(psi, r_s)
            rn = float(np.linalg.norm(r_s))
            e32 = fp32_dot_bound(n, rn, unit)
            j = int(g["idx"][s])
            best = float(np.max(np.abs(c)))
            assert abs(c[j]) >= best - (tol_sel * rn + 2 * e32), (
                f"step {s}: GPU atom {j} |c|={abs(c[j]):.6g} vs max {best:.6g}")
            coef_rel = 1e-6 if unit == U32 else 16 * unit  # FP32: the stored coefficient's rounding
            assert abs(float(g["coef"][s]) - c[j]) <= e32 + coef_rel * abs(c[j]), (
                f"step {s}: coefficient {g['coef'][s]} vs FP64 {c[j]}")
            rep.checked_after.append(int(s))

    # 4. end state of the GPU run
    if g["stop"] == "converged":
        rr = float(np.sum(g["r"].astype(np.float64) ** 2))
        assert rr <= (eps * ynorm) ** 2 * (1 + 1e-6) + 1e-30
    defect = y.astype(np.float64) - np.asarray(psi, dtype=np.float64) @ g["x"].astype(
        np.float64) - g["r"].astype(np.float64)
    assert np.linalg.norm(defect) <= max(tol, 4 * unit * np.sqrt(max(g["iters"], 1))) * max(
        ynorm, 1e-300) + 1e-30, "y != Psi x~ + r"
    if (not full and not capped and g["stop"] == "converged"
            and oracle.REASONS[ora.reason] == "converged"):
        assert abs(g["iters"] - ora.iters) <= max(8, 0.15 * ora.iters), (g["iters"], ora.iters)
    return rep
