"""The whole-run parity checker (tests/wholerun.py) on CPU decodes.

A plain FP32 Matching Pursuit written here with numpy (FP32 inner products
and updates, the smallest-index argmax) stands in for a GPU decode: the
checker must accept it, and must reject the same decode with one planted
mistake -- a wrong atom at a step whose top-two gap is large, a wrong
coefficient, a residual that drifts, or a run stopped early.
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
from wholerun import whole_run


def _fp32_mp(psi: np.ndarray, y: np.ndarray, eps: float, T: int) -> dict:
    p32 = np.asarray(psi, dtype=np.float32)
    r = np.asarray(y, dtype=np.float32).copy()
    x = np.zeros(p32.shape[1], np.float32)
    yy = float(np.sum(r.astype(np.float64) ** 2))
    idx, coef, rt = [], [], []
    stop = "max_iters"
    for _ in range(T):
        if not float(np.sum(r.astype(np.float64) ** 2)) > eps * eps * yy:
            stop = "converged"
            break
        c = p32.T @ r
        i = int(np.argmax(np.abs(c)))
        x[i] += c[i]
        r = (r - c[i] * p32[:, i]).astype(np.float32)
        idx.append(i)
        coef.append(c[i])
        rt.append(r.copy())
    else:
        if not float(np.sum(r.astype(np.float64) ** 2)) > eps * eps * yy:
            stop = "converged"
    return dict(x=x, r=r, iters=len(idx), stop=stop, idx=np.array(idx, np.int32),
                coef=np.array(coef, np.float32), r_trace=np.array(rt, np.float32))


@pytest.fixture(scope="module")
def case():
    p = mpgen.make_problem("c0", 1)
    g = _fp32_mp(p.psi, p.y, p.eps, p.max_iters)
    assert g["stop"] == "converged"
    return p, g


def test_accepts_a_correct_fp32_decode(case):
    p, g = case
    rep = whole_run(p.psi, p.y, p.eps, g)
    assert rep.steps == g["iters"] and rep.misses == 0
    assert rep.x_err < 1e-6 and rep.r_err < 1e-6


def _copy(g):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}


def test_rejects_a_wrong_atom(case):
    p, g = case
    b = _copy(g)
    b["idx"][3] = (b["idx"][3] + 1) % p.m
    with pytest.raises(AssertionError):
        whole_run(p.psi, p.y, p.eps, b)


def test_rejects_a_wrong_coefficient(case):
    p, g = case
    b = _copy(g)
    b["coef"][5] *= 1.0 + 1e-4
    with pytest.raises(AssertionError, match="coefficient"):
        whole_run(p.psi, p.y, p.eps, b)


def test_rejects_a_drifting_residual(case):
    p, g = case
    b = _copy(g)
    # every later state carries an error of 1e-4 ||y|| along one atom
    d = 1e-4 * np.linalg.norm(p.y) * p.psi[:, 7]
    b["r_trace"][20:] += d
    b["r"] = b["r"] + d
    with pytest.raises(AssertionError):
        whole_run(p.psi, p.y, p.eps, b)


def test_rejects_an_early_stop(case):
    p, g = case
    t = g["iters"] - 3
    b = dict(x=None, r=g["r_trace"][t - 1].copy(), iters=t, stop="converged",
             idx=g["idx"][:t].copy(), coef=g["coef"][:t].copy(), r_trace=g["r_trace"][:t].copy())
    xs = np.zeros(p.m, np.float32)
    for i, c in zip(b["idx"], b["coef"]):
        xs[i] += c
    b["x"] = xs
    with pytest.raises(AssertionError):
        whole_run(p.psi, p.y, p.eps, b)


def test_rejects_a_wrong_final_x(case):
    p, g = case
    b = _copy(g)
    b["x"][int(b["idx"][0])] += 1e-3
    with pytest.raises(AssertionError):
        whole_run(p.psi, p.y, p.eps, b)
