"""Exact and brute-force references used to pin the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* :func:`exact_mp` runs the MP iteration of Section 3 (eqs. 8-12) in exact
  rational arithmetic.  On dictionaries whose columns are exactly unit norm
  it gives the true index sequence, coefficients and ties, free of rounding.
* :func:`best_one_term` is the brute-force best single-atom approximation:
  for each atom it asks a least-squares solver (numpy) for the best multiple
  of that atom, and keeps the atom with the smallest residual.  For unit-norm
  atoms the greedy MP step of eqs. 9-11 is exactly this search, so it pins
  the selection rule, the coefficient and the residual update without
  reusing the MP formulas.
* :func:`best_k_support` enumerates every K-subset of atoms (the l0 problem of
  eq. 6, feasible only for tiny M) and returns the one with the smallest
  least-squares residual.
* :func:`exact_omp` runs OMP (see ``oracle.omp``) in exact rational
  arithmetic, re-fitting the selected atoms through the normal equations
  solved by Gaussian elimination on Fractions -- a different route to the
  least-squares fit than the LAPACK solver the FP64 OMP oracle uses.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np


def exact_mp(cols: Sequence[Sequence[Fraction]], y: Sequence[Fraction],
             eps: Fraction, max_iters: int):
    """MP in exact rational arithmetic.

    ``cols`` is a list of M columns (each N Fractions), ``y`` N Fractions.
    Stopping test: continue while sum r^2 > eps^2 sum y^2 and t < max_iters.
    Returns dict(idx, coef, rr, x, r, iters, reason, gap) with Fractions.
    """
    n = len(y)
    m = len(cols)
    r = [Fraction(v) for v in y]
    x = [Fraction(0)] * m
    yy = sum(v * v for v in r)
    thr = Fraction(eps) * Fraction(eps) * yy
    idx: List[int] = []
    coef: List[Fraction] = []
    rrs: List[Fraction] = []
    gaps: List[Fraction] = []
    if yy == 0:
        return dict(idx=idx, coef=coef, rr=rrs, x=x, r=r, iters=0,
                    reason="zero_input", gap=gaps)
    rr = yy
    t = 0
    while True:
        if not rr > thr:
            reason = "converged"
            break
        if t >= max_iters:
            reason = "max_iters"
            break
        c = [sum(col[i] * r[i] for i in range(n)) for col in cols]
        a = [abs(v) for v in c]
        best = max(a)
        i = a.index(best)  # first (smallest) index of the maximum
        rest = a[:i] + a[i + 1:]
        gaps.append(best - max(rest) if rest else best)
        ci = c[i]
        if ci == 0:
            reason = "stalled"
            break
        x[i] += ci
        r = [r[k] - ci * cols[i][k] for k in range(n)]
        rr = sum(v * v for v in r)
        idx.append(i)
        coef.append(ci)
        rrs.append(rr)
        t += 1
    return dict(idx=idx, coef=coef, rr=rrs, x=x, r=r, iters=t, reason=reason, gap=gaps)


def best_one_term(psi: np.ndarray, r: np.ndarray, rel_tie: float = 1e-12
                  ) -> Tuple[int, float, np.ndarray]:
    """Brute-force best approximation of r by one scaled atom.

    For every column m, ``numpy.linalg.lstsq`` gives the coefficient a_m that
    minimises ||r - a psi_m||; the atom with the smallest residual wins, the
    smallest index among residuals equal within ``rel_tie * ||r||^2``.
    Returns (index, coefficient, new residual r - a psi_index).
    """
    r = np.asarray(r, dtype=np.float64)
    n, m = psi.shape
    best = None
    for j in range(m):
        col = np.asarray(psi[:, j], dtype=np.float64).reshape(n, 1)
        a, *_ = np.linalg.lstsq(col, r, rcond=None)
        res = r - a[0] * col[:, 0]
        e = float(res @ res)
        if best is None or e < best[0] - rel_tie * float(r @ r):
            best = (e, j, float(a[0]), res)
    return best[1], best[2], best[3]


def best_k_support(psi: np.ndarray, y: np.ndarray, k: int):
    """Exhaustive l0 search (eq. 6): the K-subset with the least LS residual.

    Returns (sorted support tuple, coefficients, residual norm^2).
    """
    y = np.asarray(y, dtype=np.float64)
    a = np.asarray(psi, dtype=np.float64)
    best = None
    for sup in itertools.combinations(range(a.shape[1]), k):
        sub = a[:, list(sup)]
        coef, *_ = np.linalg.lstsq(sub, y, rcond=None)
        res = y - sub @ coef
        e = float(res @ res)
        if best is None or e < best[2]:
            best = (sup, coef, e)
    return best


def _solve_exact(a: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Solve the square system a z = b exactly (Gaussian elimination with
    the first non-zero pivot; a must be non-singular)."""
    k = len(b)
    aug = [list(a[i]) + [b[i]] for i in range(k)]
    for col in range(k):
        piv = next(r for r in range(col, k) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        for r in range(k):
            if r != col and aug[r][col] != 0:
                f = aug[r][col] / aug[col][col]
                aug[r] = [aug[r][j] - f * aug[col][j] for j in range(k + 1)]
    return [aug[i][k] / aug[i][i] for i in range(k)]


def exact_omp(cols: Sequence[Sequence[Fraction]], y: Sequence[Fraction],
              eps: Fraction, max_iters: int):
    """OMP in exact rational arithmetic (same loop, tie rule and stopping
    test as ``exact_mp``).  Returns dict(idx, coef (c_i of each selection),
    rr, x, r, iters, reason)."""
    n, m = len(y), len(cols)
    yv = [Fraction(v) for v in y]
    r = list(yv)
    yy = sum(v * v for v in yv)
    thr = Fraction(eps) * Fraction(eps) * yy
    sel: List[int] = []
    coef: List[Fraction] = []
    rrs: List[Fraction] = []
    xs: List[Fraction] = []
    if yy == 0:
        return dict(idx=sel, coef=coef, rr=rrs, x=[Fraction(0)] * m, r=r, iters=0,
                    reason="zero_input")
    rr = yy
    t = 0
    while True:
        if not rr > thr:
            reason = "converged"
            break
        if t >= max_iters:
            reason = "max_iters"
            break
        c = [sum(col[i] * r[i] for i in range(n)) for col in cols]
        a = [abs(v) for v in c]
        i = a.index(max(a))
        if c[i] == 0 or i in sel:
            reason = "stalled"
            break
        sel.append(i)
        g = [[sum(cols[p][k] * cols[q][k] for k in range(n)) for q in sel] for p in sel]
        b = [sum(cols[p][k] * yv[k] for k in range(n)) for p in sel]
        xs = _solve_exact(g, b)
        r = [yv[k] - sum(xs[j] * cols[sel[j]][k] for j in range(len(sel))) for k in range(n)]
        rr = sum(v * v for v in r)
        coef.append(c[i])
        rrs.append(rr)
        t += 1
    x = [Fraction(0)] * m
    for j, s in enumerate(sel):
        x[s] = xs[j]
    return dict(idx=sel, coef=coef, rr=rrs, x=x, r=r, iters=t, reason=reason)
