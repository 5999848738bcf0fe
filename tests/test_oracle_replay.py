"""Pins of the oracle's replay mode and of its many-vector correlation helpers
(CPU only).

The replay runs the Section 3 iteration (eqs. 10-11) with the selection of
eq. 9 replaced by a given index sequence.  It is pinned by closed forms and
stored exact values, not by re-deriving its own formula:
* orthonormal dictionaries: whatever order the support atoms are forced in,
  every coefficient is the atom's x value, x~ = x and r = 0 after the K steps,
  and the deficit of each forced atom is max_{remaining} |x_j| - |x_forced|;
* the exact rational golden fixture (written by tests/golden/make_golden.py
  from oracle/exact.py): replaying its exact index sequence on the FP64
  stereographic columns reproduces the stored exact coefficients;
* Hadamard columns with exact ties: a tied atom forced out of the eq. 16
  order has deficit exactly 0;
* replaying the free run's own sequence gives the free run back bit for bit
  with all deficits exactly 0, and a planted atom that is not a near tie is
  flagged by its deficit;
* energy: ||r_{t+1}||^2 = ||r_t||^2 - 2c^2 + c^2 ||psi||^2 and y = Psi x~ + r.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import mpgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _orthonormal_case(seed, n, k):
    rng = np.random.default_rng(seed)
    psi = mpgen.qr_orthonormal_dictionary(rng, n)
    sup = np.sort(rng.choice(n, size=k, replace=False))
    x = np.zeros(n)
    x[sup] = rng.standard_normal(k)
    return psi, x, sup, psi @ x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_orthonormal_any_order_closed_form(seed):
    """Orthonormal Psi (N = M): c_i = <Psi x - sum_{done} x_j psi_j, psi_i> = x_i
    for a support atom not yet taken, whatever the order."""
    psi, x, sup, y = _orthonormal_case(seed, 32, 7)
    order = np.random.default_rng(seed + 50).permutation(sup)
    rep = oracle.replay(psi, y, order, check_ties=True, r_trace=True, y64=True)
    np.testing.assert_allclose(rep.coef, x[order], rtol=0, atol=1e-14)
    np.testing.assert_allclose(rep.x, x, rtol=0, atol=1e-14)
    assert np.linalg.norm(rep.r) <= 1e-14 * np.linalg.norm(y)
    for t, i in enumerate(order):
        remaining = np.abs(x[order[t:]])
        assert abs(rep.deficit[t] - (remaining.max() - abs(x[i]))) <= 1e-14
    # r after step t is y minus the atoms taken so far
    for t in range(len(order)):
        part = y - psi[:, order[: t + 1]] @ x[order[: t + 1]]
        np.testing.assert_allclose(rep.r_trace[t], part, rtol=0, atol=1e-14)


def test_orthonormal_off_support_atom_has_zero_coefficient():
    psi, x, sup, y = _orthonormal_case(4, 16, 3)
    off = int(np.setdiff1d(np.arange(16), sup)[0])
    rep = oracle.replay(psi, y, [off, int(sup[0])], check_ties=True, y64=True)
    assert abs(rep.coef[0]) <= 1e-15
    assert abs(rep.deficit[0] - np.abs(x).max()) <= 1e-14
    assert abs(rep.coef[1] - x[sup[0]]) <= 1e-14


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _golden("exact_mp_stereographic.json")["cases"],
                         ids=lambda c: c["name"])
def test_replay_reproduces_exact_golden(case):
    """The stored exact rational run, replayed in FP64 on the same (exactly
    unit-norm) columns with y in FP64: coefficients and ||r||^2 within FP64
    rounding of the exact stored values, deficits 0 up to rounding."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([900, case["seed"]])))
    cols = mpgen.rational_unit_dictionary(rng, case["n"], case["m"])
    y = [sum(Fraction(c) * cols[a][i] for a, c in zip(case["atoms"], case["coefs"]))
         for i in range(case["n"])]
    psi = np.asfortranarray(np.array([[float(v) for v in c] for c in cols]).T)
    y64 = np.array([float(v) for v in y])
    rep = oracle.replay(psi, y64, case["idx"], check_ties=True, y64=True)
    exact = np.array([float(Fraction(v)) for v in case["coef"]])
    rr = np.array([float(Fraction(v)) for v in case["rr"]])
    scale = float(np.linalg.norm(y64))
    np.testing.assert_allclose(rep.coef, exact, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(rep.rr_trace, rr, rtol=0, atol=1e-13 * scale ** 2)
    gaps = np.array([float(Fraction(g)) for g in case["gap"]])
    assert np.all(rep.deficit <= 1e-14 * scale)
    assert np.all(gaps > 0)


def test_forced_tie_out_of_order_has_zero_deficit():
    """Hadamard, x with |x_3| = |x_7| = |x_11| = 1/2: forcing 11 before 3 is a
    tie (deficit exactly 0); forcing the 1/8 atom first is not (deficit 3/8)."""
    psi = mpgen.hadamard_dictionary(16)
    x = np.zeros(16, np.float32)
    x[[3, 7, 11, 12, 14, 15]] = [-0.5, 0.5, 0.5, 0.25, -0.25, 0.125]
    y = mpgen.encode(psi, x)
    rep = oracle.replay(psi, y, [11, 7, 3, 14, 12, 15])
    assert rep.deficit.tolist() == [0.0] * 6
    assert np.array_equal(rep.x, x.astype(np.float64)) and not rep.r.any()
    rep = oracle.replay(psi, y, [15, 3])
    assert rep.deficit.tolist() == [0.375, 0.0]
    assert rep.coef.tolist() == [0.125, -0.5]


@pytest.mark.parametrize("name,seed", [("c0", 0), ("c0", 1), ("c1a", 0)])
def test_replay_of_own_sequence_is_the_free_run(name, seed):
    p = mpgen.make_problem(name, seed)
    cap = p.max_iters if name == "c0" else 150
    free = oracle.solve(p.psi, p.y, p.eps, cap)
    for ties in (True, False):
        rep = oracle.replay(p.psi, p.y, free.idx, check_ties=ties)
        assert np.array_equal(rep.x, free.x) and np.array_equal(rep.r, free.r)
        assert np.array_equal(rep.coef, free.coef)
        assert np.array_equal(rep.rr_trace, free.rr_trace)
        if ties:
            assert not rep.deficit.any()


def test_planted_non_tie_index_is_flagged():
    p = mpgen.make_problem("c0", 3)
    free = oracle.solve(p.psi, p.y, p.eps, p.max_iters)
    idx = free.idx.copy()
    r5 = oracle.replay(p.psi, p.y, idx[:5], check_ties=False).r
    c = oracle.correlate(p.psi, r5)
    order = np.argsort(-np.abs(c), kind="stable")
    idx[5] = order[40]      # the 41st best atom at step 5
    rep = oracle.replay(p.psi, p.y, idx, check_ties=True)
    rn = np.sqrt(r5 @ r5)
    assert rep.deficit[5] == pytest.approx(abs(c[order[0]]) - abs(c[order[40]]), rel=1e-12)
    assert rep.deficit[5] > 1e-3 * rn
    assert not rep.deficit[:5].any()


def test_replay_energy_and_reconstruction():
    p = mpgen.make_problem("c0", 4)
    free = oracle.solve(p.psi, p.y, p.eps, p.max_iters)
    idx = free.idx.copy()
    idx[3], idx[4] = idx[4], idx[3]       # another sequence: not the free run
    rep = oracle.replay(p.psi, p.y, idx, check_ties=False)
    psi = np.asarray(p.psi, np.float64)
    nrm2 = np.sum(psi ** 2, axis=0)
    pre = np.r_[float(p.y.astype(np.float64) @ p.y.astype(np.float64)), rep.rr_trace[:-1]]
    pred = pre - 2 * rep.coef ** 2 + rep.coef ** 2 * nrm2[idx]
    assert np.all(np.abs(rep.rr_trace - pred) <= 1e-12 * pre)
    defect = p.y.astype(np.float64) - psi @ rep.x - rep.r
    assert np.linalg.norm(defect) <= 1e-13 * np.linalg.norm(p.y)


def test_replay_rejects_bad_indices():
    p = mpgen.make_problem("c0", 0)
    with pytest.raises(ValueError):
        oracle.replay(p.psi, p.y, [0, p.m])
    with pytest.raises(ValueError):
        oracle.replay(p.psi, p.y, [-1])
    rep = oracle.replay(p.psi, p.y, [])
    assert np.array_equal(rep.r, p.y.astype(np.float64)) and not rep.x.any()


# --- correlate_many / top_gap ---------------------------------------------------

def test_correlate_many_closed_form_and_sequential_sum():
    """Orthonormal Psi: Psi^T (Psi X) = X; any Psi: the sequential FP64 sum of
    ``correlate`` up to FP64 rounding."""
    rng = np.random.default_rng(7)
    q = mpgen.qr_orthonormal_dictionary(rng, 48)
    X = rng.standard_normal((48, 5))
    np.testing.assert_allclose(oracle.correlate_many(q, q @ X, chunk=2), X, rtol=0,
                               atol=1e-13)
    p = mpgen.make_problem("c0", 2)
    R = rng.standard_normal((p.n, 7)).astype(np.float32)
    C = oracle.correlate_many(p.psi, R, chunk=3)
    for j in range(R.shape[1]):
        c = oracle.correlate(p.psi, R[:, j])
        assert np.max(np.abs(C[:, j] - c)) <= 1e-13 * np.linalg.norm(R[:, j])


def test_top_gap_brute_force():
    rng = np.random.default_rng(8)
    C = rng.standard_normal((37, 9))
    C[5, 0], C[2, 0] = 9.0, -9.0      # exact tie of |c|: smallest index wins, gap 0
    C[:, 1] = 0.0                     # all zero: index 0, gap 0
    C[30, 2] = 50.0
    best, top, gap = oracle.top_gap(C)
    for j in range(C.shape[1]):
        a = [abs(v) for v in C[:, j]]
        srt = sorted(range(len(a)), key=lambda i: (-a[i], i))
        assert best[j] == srt[0]
        assert top[j] == a[srt[0]]
        assert gap[j] == a[srt[0]] - a[srt[1]]
    assert best[0] == 2 and gap[0] == 0.0 and best[1] == 0 and best[2] == 30
    b1, t1, g1 = oracle.top_gap(np.array([[-3.0, 2.0]]))
    assert b1.tolist() == [0, 0] and g1.tolist() == [3.0, 2.0]
