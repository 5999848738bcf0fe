"""Pins of the FP64 OMP oracle (``oracle.omp``) against facts fixed by the
definition and by mathematics, and planted mistakes that the pins must catch.

OMP keeps MP's selection (eq. 9, tie rule of eq. 16) and re-fits all selected
atoms by least squares after each selection.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import mpgen
import oracle
from oracle import omp
from oracle.exact import exact_omp


def _gauss_unit(seed, n, m):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, m))
    return np.asfortranarray(g / np.linalg.norm(g, axis=0))


def _sparse(seed, m, k):
    rng = np.random.default_rng(seed + 77)
    sup = np.sort(rng.choice(m, size=k, replace=False))
    x = np.zeros(m)
    x[sup] = rng.uniform(0.5, 1.5, size=k) * np.where(rng.random(k) < 0.5, -1, 1)
    return x, sup


# ---- facts ---------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_orthonormal_dictionary_omp_is_mp(seed):
    """With orthonormal columns the least-squares re-fit changes nothing: OMP
    takes exactly MP's steps (compared with the pinned MP oracle)."""
    rng = np.random.default_rng(500 + seed)
    q = mpgen.qr_orthonormal_dictionary(rng, 48)
    x = np.zeros(48)
    sup = rng.choice(48, size=7, replace=False)
    x[sup] = rng.standard_normal(7)
    y = q @ x
    a = omp.solve_omp(q, y, 1e-10, 40, y_dtype=np.float64)
    b = oracle.solve64(q, y, 1e-10, 40)
    assert a.iters == b.iters == 7
    assert a.idx.tolist() == b.idx.tolist()
    np.testing.assert_allclose(a.x, b.x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_rational_omp(seed):
    """Exactly unit-norm rational columns, a 3-sparse rational x: exact OMP
    (normal equations on Fractions) and the FP64 oracle take the same atoms
    in the same order, and their fitted x~ agree to FP64 rounding.  (With
    N = 6 < M = 10 OMP may reach r = 0 on a support other than x's.)"""
    rng = np.random.default_rng(40 + seed)
    n, m, k = 6, 10, 3
    cols = mpgen.rational_unit_dictionary(rng, n, m)
    sup = sorted(rng.choice(m, size=k, replace=False).tolist())
    xq = [Fraction(0)] * m
    for j, s in enumerate(sup):
        xq[s] = Fraction(int(rng.integers(3, 9)) * (1 if j % 2 else -1), 4)
    yq = [sum(xq[s] * cols[s][i] for s in sup) for i in range(n)]
    ex = exact_omp(cols, yq, Fraction(1, 10 ** 9), 10)
    psi = np.array([[float(v) for v in col] for col in cols]).T.copy(order="F")
    y = np.array([float(v) for v in yq])
    fp = omp.solve_omp(psi, y, 1e-9, 10, y_dtype=np.float64)
    assert ex["iters"] >= 1 and ex["reason"] == "converged"
    assert fp.idx.tolist() == ex["idx"] and fp.iters == ex["iters"]
    np.testing.assert_allclose(fp.x, [float(v) for v in ex["x"]], rtol=0, atol=1e-12)
    np.testing.assert_allclose(fp.coef, [float(v) for v in ex["coef"]], rtol=1e-13, atol=1e-15)


def test_tie_goes_to_smallest_index():
    """Hadamard columns (orthonormal, entries +-1/4) and two nonzeros of equal
    magnitude: the correlations are exact dyadic values, |c| ties exactly,
    and the smaller index is taken first (eq. 16)."""
    psi = mpgen.hadamard_dictionary(16).astype(np.float64)
    x = np.zeros(16)
    x[[9, 3, 12]] = [-0.5, 0.5, 0.25]
    res = omp.solve_omp(psi, psi @ x, 1e-12, 10, y_dtype=np.float64)
    assert res.idx.tolist() == [3, 9, 12] and res.reason == omp.CONVERGED
    np.testing.assert_allclose(res.x, x, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_recovers_sparse_signal_in_k_steps(seed):
    """N=64, M=128, K=5 (mutual coherence small enough that OMP succeeds):
    exactly K steps, x~ = x to FP64 rounding, r ~ 0."""
    psi = _gauss_unit(seed, 64, 128)
    x, sup = _sparse(seed, 128, 5)
    y = psi @ x
    res = omp.solve_omp(psi, y, 1e-10, 100, y_dtype=np.float64)
    assert res.iters == 5 and res.reason == omp.CONVERGED
    assert sorted(res.idx.tolist()) == sup.tolist()
    assert np.linalg.norm(res.x - x) <= 1e-12 * np.linalg.norm(x)


def test_residual_is_orthogonal_to_selected_atoms():
    """After every step r is orthogonal to all selected atoms (the least-
    squares normal equations), and ||y||^2 = ||r||^2 + ||Psi_S x_S||^2."""
    psi = _gauss_unit(9, 80, 200)
    x, _ = _sparse(9, 200, 12)
    y = psi @ x
    yy = float(y @ y)
    for t in range(1, 13):
        res = omp.solve_omp(psi, y, 0.0, t, y_dtype=np.float64)
        ps = psi[:, res.idx]
        assert np.max(np.abs(ps.T @ res.r)) <= 1e-12 * np.sqrt(yy)
        fit = ps @ res.x[res.idx]
        assert abs(yy - (res.r @ res.r + fit @ fit)) <= 1e-12 * yy
    full = omp.solve_omp(psi, y, 0.0, 12, y_dtype=np.float64)
    assert np.all(np.diff(full.rr_trace) <= 1e-12 * yy)


def test_stop_rules():
    psi = _gauss_unit(3, 32, 64)
    x, _ = _sparse(3, 64, 4)
    y = psi @ x
    assert omp.solve_omp(psi, np.zeros(32), 1e-6, 10).reason == omp.ZERO_INPUT
    r0 = omp.solve_omp(psi, y, 1e-6, 0, y_dtype=np.float64)
    assert r0.iters == 0 and r0.reason == omp.MAX_ITERS
    r2 = omp.solve_omp(psi, y, 1e-6, 2, y_dtype=np.float64)
    assert r2.iters == 2 and r2.reason == omp.MAX_ITERS
    assert omp.solve_omp(psi, y, 2.0, 10, y_dtype=np.float64).iters == 0
    # a dictionary with a zero column and y orthogonal to every other column
    z = np.zeros((4, 2))
    z[0, 1] = 1.0
    st = omp.solve_omp(np.asfortranarray(z), np.array([0.0, 1.0, 0.0, 0.0]), 1e-6, 5,
                       y_dtype=np.float64)
    assert st.reason == omp.STALLED and st.iters == 0


# ---- planted mistakes ----------------------------------------------------------

def _battery():
    failed = []
    try:
        test_orthonormal_dictionary_omp_is_mp(0)
    except AssertionError:
        failed.append("orthonormal")
    try:
        test_tie_goes_to_smallest_index()
    except AssertionError:
        failed.append("tie")
    try:
        for s in range(3):
            test_recovers_sparse_signal_in_k_steps(s)
    except AssertionError:
        failed.append("recovery")
    try:
        test_residual_is_orthogonal_to_selected_atoms()
    except AssertionError:
        failed.append("orthogonality")
    return failed


def test_unmodified_omp_passes_battery():
    assert _battery() == []


def _signed_argmax(c):
    i = int(np.argmax(c))
    return i, 0.0


def _largest_index_tie(c):
    a = np.abs(c)
    i = int(len(a) - 1 - np.argmax(a[::-1]))
    return i, 0.0


def _no_refit(psi_s, y):  # MP-like: only the newest coefficient, others frozen at 0
    z = np.zeros(psi_s.shape[1])
    z[-1] = psi_s[:, -1] @ y
    return z


def _residual_sign(y, psi_s, xs):
    return y + psi_s @ xs


@pytest.mark.parametrize("name,attr,fn", [
    ("signed_argmax", "_argmax_abs", _signed_argmax),
    ("tie_to_largest_index", "_argmax_abs", _largest_index_tie),
    ("no_refit", "_fit", _no_refit),
    ("residual_sign", "_residual", _residual_sign),
])
def test_planted_mistakes_are_caught(monkeypatch, name, attr, fn):
    monkeypatch.setattr(omp, attr, fn)
    with np.errstate(all="ignore"):
        assert _battery(), f"mutant {name} passed every pin"
