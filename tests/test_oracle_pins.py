"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test names the passage it follows.  Together they are chosen so that a
plausible slip in the oracle -- argmax of c instead of |c|, a wrong sign in the
coefficient or the residual update, a transposed dictionary, a wrong tie rule,
an off-by-one in the stopping test -- fails at least one of them
(``test_planted_mistakes_are_caught`` checks that on purpose-built mutants).
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import mpgen
import oracle
from oracle.exact import best_k_support, best_one_term, exact_mp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit_gaussian_f64(seed, n, m):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, m))
    return np.asfortranarray(g / np.linalg.norm(g, axis=0))


def _sparse_y(psi, seed, k):
    rng = np.random.default_rng(seed + 1000)
    m = psi.shape[1]
    sup = np.sort(rng.choice(m, size=k, replace=False))
    x = np.zeros(m)
    x[sup] = rng.standard_normal(k)
    y = (np.asarray(psi, dtype=np.float64) @ x).astype(np.float32)
    return x, sup, y


# --- worked examples (hand-derived, eq. 16 tie rule) ------------------------

def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _golden("hadamard_ties.json")["cases"], ids=lambda c: c["name"])
def test_hadamard_tie_golden(case):
    """Section 3 loop + eq. 16: equal |c| are taken smallest index first."""
    psi = mpgen.hadamard_dictionary(case["n"])
    x = np.zeros(case["n"], dtype=np.float32)
    for k, v in case["x"].items():
        x[int(k)] = v
    y = mpgen.encode(psi, x)
    res = oracle.solve(psi, y, case["eps"], case["max_iters"])
    assert res.iters == case["iters"]
    assert oracle.REASONS[res.reason] == case["reason"]
    assert res.idx.tolist() == case["idx"]
    assert res.coef.tolist() == case["coef"]          # exact: dyadic arithmetic
    assert res.rr_trace.tolist() == case["rr"]
    if case["reason"] == "converged" and case["eps"] == 0.0:
        assert np.array_equal(res.x, x.astype(np.float64))


# --- exact rational arithmetic ----------------------------------------------

def _rational_case(seed, n, m, atoms, coefs):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([900, seed])))
    cols = mpgen.rational_unit_dictionary(rng, n, m)
    y = [sum(Fraction(c) * cols[a][i] for a, c in zip(atoms, coefs)) for i in range(n)]
    return cols, y


@pytest.mark.parametrize("case", _golden("exact_mp_stereographic.json")["cases"],
                         ids=lambda c: c["name"])
def test_exact_rational_golden(case):
    """FP64 oracle vs exact rational MP (Section 3) on exactly unit-norm columns."""
    cols, y = _rational_case(case["seed"], case["n"], case["m"], case["atoms"], case["coefs"])
    psi = np.asfortranarray(np.array([[float(v) for v in c] for c in cols]).T)
    y64 = np.array([float(v) for v in y])
    # the oracle takes FP32 y; these y are not FP32-exact, so compare against an
    # exact run on the FP32-rounded y as well as the stored sequence
    y32 = y64.astype(np.float32)
    res = oracle.solve(psi, y32, 0.0, case["iters"])
    ex = exact_mp(cols, [Fraction(float(v)) for v in y32], Fraction(0), case["iters"])
    assert res.idx.tolist() == ex["idx"]
    ycoef = np.array([float(v) for v in ex["coef"]])
    np.testing.assert_allclose(res.coef, ycoef, rtol=1e-12, atol=1e-13 * np.linalg.norm(y64))
    # the stored fixture (exact y) must select the same atoms while gaps are clear
    stored = case["idx"]
    gaps = [float(Fraction(g)) for g in case["gap"]]
    for t, (a, b) in enumerate(zip(res.idx.tolist(), stored)):
        if gaps[t] < 1e-6:
            break
        assert a == b, f"step {t}"


@pytest.mark.parametrize("seed", range(6))
def test_exact_rational_random(seed):
    """Live exact-vs-FP64 comparison on random rational dictionaries."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([901, seed])))
    n, m = 5 + seed % 3, 9 + seed
    cols = mpgen.rational_unit_dictionary(rng, n, m)
    yv = rng.integers(-9, 10, size=n) / 8.0  # dyadic: exact in FP32
    y = [Fraction(float(v)) for v in yv]
    ex = exact_mp(cols, y, Fraction(1, 10 ** 6), 10)
    psi = np.asfortranarray(np.array([[float(v) for v in c] for c in cols]).T)
    res = oracle.solve(psi, yv.astype(np.float32), 1e-6, 10)
    gaps = [float(g) for g in ex["gap"]]
    k = next((t for t, g in enumerate(gaps) if g < 1e-9), len(ex["idx"]))
    assert res.idx.tolist()[:k] == ex["idx"][:k]
    np.testing.assert_allclose(res.coef[:k], [float(v) for v in ex["coef"][:k]],
                               rtol=1e-12, atol=1e-14)
    if k == len(ex["idx"]):
        assert res.iters == ex["iters"]
        np.testing.assert_allclose(res.x, [float(v) for v in ex["x"]], atol=1e-13)


# --- brute force: MP's step is the best one-term approximation ---------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_each_step_is_best_one_term(seed):
    """Eqs. 9-11 with unit-norm columns = exhaustive best single-atom fit."""
    n, m, steps = 24, 40, 12
    psi = _unit_gaussian_f64(seed, n, m)
    _, _, y = _sparse_y(psi, seed, 4)
    full = oracle.solve(psi, y, 0.0, steps)
    r = y.astype(np.float64)
    for t in range(steps):
        j, a, r_bf = best_one_term(psi, r)
        assert full.idx[t] == j
        assert abs(full.coef[t] - a) <= 1e-12 * np.linalg.norm(r)
        part = oracle.solve(psi, y, 0.0, t + 1)
        np.testing.assert_allclose(part.r, r_bf, rtol=0, atol=1e-12 * np.linalg.norm(y))
        r = r_bf


def test_argmax_is_on_magnitude():
    """Eq. 9 maximises |<r, psi>|: a large negative correlation must win."""
    psi = np.asfortranarray(np.eye(3))
    y = np.array([0.5, -0.9, 0.7], dtype=np.float32)
    res = oracle.solve(psi, y, 0.0, 1)
    assert res.idx.tolist() == [1]
    assert res.coef[0] == pytest.approx(-0.9, abs=1e-7)


# --- orthonormal dictionaries: MP reduces to sorting |Psi^T y| ---------------

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_orthonormal_qr_is_sort(seed):
    """N = M orthonormal: c = x, so MP takes the support by |x| descending and
    stops after exactly K steps with x~ = x (textbook reduction; order from
    numpy's stable argsort)."""
    n, k = 64, 8
    rng = np.random.default_rng(100 + seed)
    q = mpgen.qr_orthonormal_dictionary(rng, n)
    sup = np.sort(rng.choice(n, size=k, replace=False))
    x = np.zeros(n)
    x[sup] = rng.standard_normal(k)
    y32 = (q @ x).astype(np.float32)
    # rounding y to FP32 leaves ~1e-8 relative noise on every coefficient, far
    # below eps = 1e-6, so exactly the K support atoms are taken
    c0 = q.T @ y32.astype(np.float64)
    res = oracle.solve(q, y32, 1e-6, 100)
    order = sup[np.argsort(-np.abs(c0[sup]), kind="stable")]
    assert res.iters == k
    assert res.reason == oracle.CONVERGED
    assert res.idx.tolist() == order.tolist()
    expect = np.zeros(n)
    expect[sup] = c0[sup]
    np.testing.assert_allclose(res.x, expect, rtol=0, atol=1e-14 * np.linalg.norm(x))


def test_orthonormal_hadamard_exact():
    n = 256
    psi = mpgen.hadamard_dictionary(n)
    rng = np.random.default_rng(7)
    sup = np.sort(rng.choice(n, size=12, replace=False))
    x = np.zeros(n, dtype=np.float32)
    x[sup] = rng.integers(1, 64, size=12) * np.where(rng.random(12) < 0.5, -1, 1) / 64.0
    y = mpgen.encode(psi, x)
    res = oracle.solve(psi, y, 0.0, 100)
    assert res.iters == 12 and res.rr == 0.0
    assert np.array_equal(res.x, x.astype(np.float64))
    order = sup[np.argsort(-np.abs(x[sup]), kind="stable")]
    assert res.idx.tolist() == order.tolist()


# --- the FP64-y entry point (inputs of the FP64 decode) ----------------------

def test_solve64_equals_solve_when_y_is_fp32():
    """With y exactly representable in FP32 both entry points run the same
    FP64 arithmetic (the FP64 entry only skips the rounding of y)."""
    psi = _unit_gaussian_f64(5, 48, 96)
    _, _, y = _sparse_y(psi, 6, 5)
    a = oracle.solve(psi, y, 1e-9, 60)
    b = oracle.solve64(psi, y.astype(np.float64), 1e-9, 60)
    assert a.iters == b.iters and a.reason == b.reason
    assert np.array_equal(a.idx, b.idx) and np.array_equal(a.coef, b.coef)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.r, b.r)


@pytest.mark.parametrize("seed", [0, 1])
def test_solve64_orthonormal_keeps_fp64_y(seed):
    """N = M orthonormal FP64 dictionary and FP64 nonzeros: MP is the sort of
    |x| and recovers x to FP64 rounding in exactly K steps (textbook
    reduction).  Rounding y to FP32 would leave errors of order 1e-8."""
    n, k = 64, 8
    rng = np.random.default_rng(300 + seed)
    q = mpgen.qr_orthonormal_dictionary(rng, n)
    sup = np.sort(rng.choice(n, size=k, replace=False))
    x = np.zeros(n)
    x[sup] = rng.standard_normal(k)
    y = q @ x
    res = oracle.solve64(q, y, 1e-12, 100)
    c0 = q.T @ y
    order = sup[np.argsort(-np.abs(c0[sup]), kind="stable")]
    assert res.iters == k and res.reason == oracle.CONVERGED
    assert res.idx.tolist() == order.tolist()
    assert np.linalg.norm(res.x - x) <= 1e-14 * np.linalg.norm(x)


def test_solve64_dyadic_exact():
    """Hadamard columns (entries +-1/4) and dyadic nonzeros that need more
    than FP32's 24 significant bits: every step is exact in FP64, so x~ = x
    and r = 0 exactly after K steps, largest |x| first."""
    psi = mpgen.hadamard_dictionary(16).astype(np.float64)
    x = np.zeros(16)
    x[[1, 4, 9]] = [0.5 + 2.0 ** -30, -(0.25 + 2.0 ** -40), 0.125 + 2.0 ** -35]
    y = psi @ x
    res = oracle.solve64(psi, y, 0.0, 10)
    assert res.idx.tolist() == [1, 4, 9] and res.reason == oracle.CONVERGED
    assert np.array_equal(res.x, x) and res.rr == 0.0 and not np.any(res.r)


# --- invariants --------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_energy_identity_unit_columns(seed):
    """||r_{k+1}||^2 = ||r_k||^2 - c_k^2 for unit-norm columns (eq. 11 with
    eq. 4), relative to the pre-step norm, 1e-12; telescoped: ||y||^2 =
    ||r_t||^2 + sum c^2."""
    psi = _unit_gaussian_f64(seed, 128, 512)
    _, _, y = _sparse_y(psi, seed, 10)
    res = oracle.solve(psi, y, 1e-7, 400)
    pre = np.r_[res.yy, res.rr_trace[:-1]]
    pred = pre - res.coef ** 2
    assert np.all(np.abs(res.rr_trace - pred) <= 1e-12 * pre)
    assert abs(res.yy - res.rr - np.sum(res.coef ** 2)) <= 1e-12 * res.yy
    assert np.all(np.diff(np.r_[res.yy, res.rr_trace]) <= 0)


def test_energy_identity_fp32_columns():
    """General form for columns that are unit norm only to FP32 rounding:
    ||r - c psi||^2 = ||r||^2 - 2c^2 + c^2 ||psi||^2."""
    p = mpgen.make_problem("c0", 0)
    res = oracle.solve(p.psi, p.y, p.eps, p.max_iters)
    nrm2 = np.sum(np.asarray(p.psi, dtype=np.float64) ** 2, axis=0)
    pre = np.r_[res.yy, res.rr_trace[:-1]]
    c = res.coef
    pred = pre - 2 * c ** 2 + c ** 2 * nrm2[res.idx]
    assert np.all(np.abs(res.rr_trace - pred) <= 1e-12 * pre)


@pytest.mark.parametrize("name,seed", [("c0", 0), ("c0", 1), ("c0", 2)])
def test_reconstruction_invariant(name, seed):
    """y = Psi x~ + r holds along the whole run (eqs. 10-11 move the same
    amount between x~ and r), to FP64 rounding."""
    p = mpgen.make_problem(name, seed)
    res = oracle.solve(p.psi, p.y, p.eps, p.max_iters)
    psi64 = np.asarray(p.psi, dtype=np.float64)
    defect = p.y.astype(np.float64) - psi64 @ res.x - res.r
    assert np.linalg.norm(defect) <= 1e-13 * np.linalg.norm(p.y)
    assert res.reason == oracle.CONVERGED
    assert res.rr <= p.eps ** 2 * res.yy


def test_used_atom_has_zero_correlation_next():
    """<r - c psi, psi> = c (1 - ||psi||^2) = 0 for a unit column."""
    psi = _unit_gaussian_f64(5, 50, 120)
    _, _, y = _sparse_y(psi, 5, 6)
    for t in range(1, 8):
        part = oracle.solve(psi, y, 0.0, t)
        c = oracle.correlate(psi, part.r)
        assert abs(c[part.idx[-1]]) <= 1e-13 * np.sqrt(part.yy)


def test_correlate_matches_blas():
    """The FP64 inner products agree with numpy's GEMV (a library routine)."""
    p = mpgen.make_problem("c0", 3)
    r = np.random.default_rng(0).standard_normal(p.n)
    c = oracle.correlate(p.psi, r)
    ref = np.asarray(p.psi, dtype=np.float64).T @ r
    np.testing.assert_allclose(c, ref, rtol=0, atol=1e-12 * np.linalg.norm(r))


# --- stopping rule (step 2 of the pseudo-code) ------------------------------

def test_stop_zero_iterations_cap():
    p = mpgen.make_problem("c0", 0)
    res = oracle.solve(p.psi, p.y, p.eps, 0)
    assert res.iters == 0 and res.reason == oracle.MAX_ITERS
    assert np.array_equal(res.r, p.y.astype(np.float64)) and not res.x.any()


def test_stop_eps_one_is_immediate():
    p = mpgen.make_problem("c0", 0)
    res = oracle.solve(p.psi, p.y, 1.0, 10)
    assert res.iters == 0 and res.reason == oracle.CONVERGED


def test_zero_input():
    p = mpgen.make_problem("c0", 0)
    res = oracle.solve(p.psi, np.zeros(p.n, np.float32), p.eps, 10)
    assert res.iters == 0 and res.reason == oracle.ZERO_INPUT and not res.x.any()


def test_stalled_when_no_atom_correlates():
    psi = np.asfortranarray(np.array([[1.0, 1.0, -1.0], [0.0, 0.0, 0.0]], dtype=np.float32))
    res = oracle.solve(psi, np.array([0.0, 1.0], np.float32), 0.0, 5)
    assert res.iters == 0 and res.reason == oracle.STALLED


def test_stop_count_orthonormal():
    """Orthonormal case: after k steps ||r||^2 is the sum of the squares of the
    entries still unselected, so eps between two consecutive tails fixes the
    stop count exactly."""
    n = 64
    q = mpgen.qr_orthonormal_dictionary(np.random.default_rng(11), n)
    x = np.zeros(n)
    x[[5, 17, 30, 41, 60]] = [4.0, -3.0, 2.0, 1.0, 0.5]
    y = (q @ x).astype(np.float32)
    tails = [np.sum(np.sort(np.abs(x))[::-1][k:] ** 2) for k in range(6)]
    yy = tails[0]
    for k in range(1, 5):
        eps = np.sqrt(0.5 * (tails[k] + tails[k - 1]) / yy)
        res = oracle.solve(q, y, eps, 100)
        assert res.iters == k, (k, res.iters)


def test_thread_count_does_not_change_results():
    p = mpgen.make_problem("c0", 1)
    n0 = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        a = oracle.solve(p.psi, p.y, p.eps, p.max_iters)
    finally:
        oracle.set_num_threads(n0)
    b = oracle.solve(p.psi, p.y, p.eps, p.max_iters)
    assert np.array_equal(a.idx, b.idx) and np.array_equal(a.x, b.x)
    assert np.array_equal(a.r, b.r)


def test_rejects_bad_arguments():
    p = mpgen.make_problem("c0", 0)
    with pytest.raises(ValueError):
        oracle.solve(p.psi, p.y, -1.0, 10)
    with pytest.raises(ValueError):
        oracle.solve(p.psi, p.y, p.eps, -1)


# --- recovery (eq. 6 brute force; statistical claim of Section 3) ------------

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_recovery_matches_l0_search_at_large_rho(seed):
    """At large rho MP recovers the K-sparse x (Section 3's experiment): the K
    largest |x~| sit on the l0 optimum found by exhaustive search (eq. 6)."""
    n, m, k = 12, 16, 2
    psi = _unit_gaussian_f64(40 + seed, n, m)
    x, sup, y = _sparse_y(psi, 40 + seed, k)
    l0_sup, _, e = best_k_support(psi, y, k)
    assert tuple(sup.tolist()) == l0_sup and e < 1e-10
    res = oracle.solve(psi, y, 1e-7, 2000)
    top = np.sort(np.argsort(-np.abs(res.x))[:k])
    assert top.tolist() == sup.tolist()
    err = np.sum((res.x - x) ** 2) / np.sum(x ** 2)   # eq. 14 without the 100%
    assert err < 1e-8
