"""The seeded input generators: determinism and the workload recipe."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen


def test_same_seed_same_problem():
    a = mpgen.make_problem("c0", 3)
    b = mpgen.make_problem("c0", 3)
    assert np.array_equal(a.psi, b.psi) and np.array_equal(a.y, b.y)
    assert np.array_equal(a.support, b.support)
    c = mpgen.make_problem("c0", 4)
    assert not np.array_equal(a.psi, c.psi)


@pytest.mark.parametrize("name", ["c0", "c1a"])
def test_problem_recipe(name):
    w = mpgen.workload(name)
    p = mpgen.make_problem(name, 0)
    assert p.psi.shape == (w["n"], w["m"]) and p.psi.dtype == np.float32
    assert p.psi.flags.f_contiguous
    norms = np.linalg.norm(np.asarray(p.psi, dtype=np.float64), axis=0)
    assert np.all(np.abs(norms - 1.0) < 1e-6)
    assert len(np.unique(p.support)) == w["k"] == np.count_nonzero(p.x)
    y64 = np.asarray(p.psi, dtype=np.float64)[:, p.support] @ p.x[p.support].astype(np.float64)
    assert np.array_equal(p.y, y64.astype(np.float32))
    assert p.eps == w["eps"] and p.max_iters == w["max_iters"]


def test_loguniform_values():
    p = mpgen.make_problem("c0", 0, dist="loguniform")
    v = np.abs(p.x[p.support])
    assert np.all((v >= 1e-3 * (1 - 1e-6)) & (v <= 1.0))


def test_given_dictionary_gives_the_same_problem():
    """A dictionary drawn by an earlier call, passed back in, yields exactly
    the problem a fresh draw gives (for the other value law too)."""
    a = mpgen.make_problem("c0", 2)
    for dist in ("normal", "loguniform"):
        fresh = mpgen.make_problem("c0", 2, dist=dist)
        reuse = mpgen.make_problem("c0", 2, dist=dist, psi=a.psi)
        assert np.array_equal(fresh.psi, reuse.psi) and np.array_equal(fresh.y, reuse.y)
        assert np.array_equal(fresh.x, reuse.x) and np.array_equal(fresh.support, reuse.support)
    with pytest.raises(ValueError):
        mpgen.make_problem("c0", 2, psi=np.ascontiguousarray(a.psi))


def test_batch_recipe():
    bt = mpgen.make_batch(0, b=8, n=64, m=256, kmin=2, kmax=6)
    assert bt.x.shape == (256, 8) and bt.y.shape == (64, 8)
    assert np.all((bt.k >= 2) & (bt.k <= 6))
    for j in range(8):
        assert np.count_nonzero(bt.x[:, j]) == bt.k[j]
        sup = np.flatnonzero(bt.x[:, j])
        y = mpgen.encode(bt.psi, bt.x[:, j], sup)
        assert np.array_equal(y, bt.y[:, j])
    assert np.array_equal(bt.max_iters, 20 * bt.k)


def test_ragged_recipe():
    probs = mpgen.make_ragged(0, count=6, n_choices=(16, 32))
    assert len(probs) == 6
    for p in probs:
        assert p.n in (16, 32) and p.m == 4 * p.n
        assert len(p.support) == p.n // 16


def test_hadamard_orthonormal():
    h = mpgen.hadamard_dictionary(64).astype(np.float64)
    assert np.array_equal(h.T @ h, np.eye(64))


def test_rational_columns_exact_unit_norm():
    rng = np.random.default_rng(0)
    cols = mpgen.rational_unit_dictionary(rng, 5, 7)
    for c in cols:
        assert sum(v * v for v in c) == 1


def test_fp64_problem_is_the_fp32_problem_unrounded():
    p32 = mpgen.make_problem("c0", 3)
    p64 = mpgen.make_problem("c0", 3, precision="f64")
    assert p64.psi.dtype == np.float64 and p64.psi.flags.f_contiguous
    assert np.array_equal(p64.psi.astype(np.float32), p32.psi)
    assert np.array_equal(p64.support, p32.support)
    assert np.array_equal(p64.x.astype(np.float32), p32.x)
    assert np.abs(np.linalg.norm(p64.psi, axis=0) - 1.0).max() < 1e-14
    np.testing.assert_allclose(p64.y, p64.psi[:, p64.support] @ p64.x[p64.support],
                               rtol=0, atol=1e-13)
    assert p64.y.dtype == np.float64


def test_phase_batch_follows_the_experiment():
    """Fig. 1 inputs: Bernoulli +-1/sqrt(N) columns (eq. 13), K = sigma M
    nonzeros from U[-1, 1], y = psi x."""
    sig = [0.01, 0.1, 0.5]
    pb = mpgen.make_phase_batch(0, 0.2, sig, draw=1, per_sigma=3)
    n, m = pb.psi.shape
    assert (n, m) == (200, 1000) and pb.max_iters == n and pb.eps == 1e-7
    v = np.float32(1.0 / np.sqrt(n))
    assert set(np.unique(np.abs(pb.psi))) == {v}
    assert pb.ks.tolist() == [10, 10, 10, 100, 100, 100, 500, 500, 500]
    for j in range(pb.x.shape[1]):
        nz = np.flatnonzero(pb.x[:, j])
        assert len(nz) == pb.ks[j] and np.all(np.abs(pb.x[nz, j]) <= 1.0)
    np.testing.assert_allclose(pb.y, (pb.psi.astype(np.float64) @ pb.x.astype(np.float64)),
                               rtol=0, atol=1e-6)
    again = mpgen.make_phase_batch(0, 0.2, sig, draw=1, per_sigma=3)
    assert np.array_equal(again.y, pb.y)
    other = mpgen.make_phase_batch(0, 0.2, sig, draw=2, per_sigma=3)
    assert not np.array_equal(other.psi, pb.psi)
