"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each mutant is the oracle's C source with one plausible slip substituted in,
compiled with gcc to a temporary library.  The pin battery below (the same
facts as ``test_oracle_pins.py``: hand-derived ties, best one-term fits,
energy bookkeeping, reconstruction, stop counts) must fail on every mutant and
pass on the unmodified source.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import mpgen
import oracle
from oracle import build as obuild
from oracle.exact import best_one_term

SRC = obuild.SRC

MUTANTS = {
    "signed_argmax": ("double a = fabs(c[j]);", "double a = c[j];"),
    "tie_to_largest_index": ("if (a > b) {", "if (a >= b) {"),
    "update_sign": ("r_out[k] -= ci * (double)col[k];", "r_out[k] += ci * (double)col[k];"),
    "coef_assign_not_accumulate": ("x_out[i] += ci;", "x_out[i] = ci;"),
    "eps_not_squared": ("const double thr = eps * eps * yy;", "const double thr = eps * yy;"),
    "cap_off_by_one": ("if (t >= max_iters)", "if (t > max_iters)"),
    "dropped_last_term": ("for (int64_t i = 0; i < n; ++i) s += (double)col[i] * r[i];",
                          "for (int64_t i = 0; i + 1 < n; ++i) s += (double)col[i] * r[i];"),
    "stale_norm": ("rr = sumsq(r_out, n);", "rr = rr - ci * ci * 0.5;"),
    # the replay mode
    "replay_deficit_signed": ("deficit = best - fabs(ci);", "deficit = best - ci;"),
    "replay_coef_from_y": ("for (int64_t k = 0; k < n; ++k) s += (double)col[k] * r_out[k];",
                           "for (int64_t k = 0; k < n; ++k) s += (double)col[k] * (double)y[k];"),
    "replay_deficit_vs_second": ("(void)argmax_abs(c, m, &best, &second);",
                                 "(void)argmax_abs(c, m, &second, &best);"),
}


def _build_variant(tmp_path, name, sub):
    src = open(SRC).read()
    old, new = sub
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    out = str(tmp_path / f"lib_{name}.so")
    obuild.build(src=str(path), out=out)
    return oracle.load_library(out)


def _pin_battery(lib):
    """Return the list of pins that fail for this compiled oracle."""
    with np.errstate(all="ignore"):   # mutants may overflow; that is a failure too
        return _run_battery(lib)


def _run_battery(lib):
    failed = []
    # 1. hand-derived Hadamard tie example (eq. 16)
    psi = mpgen.hadamard_dictionary(16)
    x = np.zeros(16, np.float32)
    x[[3, 7, 11, 12, 14, 15]] = [-0.5, 0.5, 0.5, 0.25, -0.25, 0.125]
    y = mpgen.encode(psi, x)
    res = oracle.solve(psi, y, 0.0, 20, lib=lib)
    if res.idx.tolist() != [3, 7, 11, 12, 14, 15] or not np.array_equal(res.x, x.astype(float)):
        failed.append("hadamard_ties")
    # 2. each step is the best one-term fit (brute force through lstsq)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((24, 40))
    psi64 = np.asfortranarray(g / np.linalg.norm(g, axis=0))
    xs = np.zeros(40)
    xs[[2, 9, 33]] = [1.0, -2.0, 0.5]
    y2 = (psi64 @ xs).astype(np.float32)
    full = oracle.solve(psi64, y2, 0.0, 10, lib=lib)
    r = y2.astype(np.float64)
    for t in range(min(10, full.iters)):
        j, a, r = best_one_term(psi64, r)
        if full.idx[t] != j or abs(full.coef[t] - a) > 1e-12:
            failed.append("best_one_term")
            break
    if full.iters != 10:
        failed.append("best_one_term_iters")
    # 3. energy identity and reconstruction on a real workload
    p = mpgen.make_problem("c0", 0)
    res = oracle.solve(p.psi, p.y, p.eps, p.max_iters, lib=lib)
    psi32 = np.asarray(p.psi, dtype=np.float64)
    defect = p.y.astype(np.float64) - psi32 @ res.x - res.r
    if np.linalg.norm(defect) > 1e-13 * np.linalg.norm(p.y):
        failed.append("reconstruction")
    if res.iters:
        nrm2 = np.sum(psi32 ** 2, axis=0)
        pre = np.r_[res.yy, res.rr_trace[:-1]]
        pred = pre - 2 * res.coef ** 2 + res.coef ** 2 * nrm2[res.idx]
        if np.any(np.abs(res.rr_trace - pred) > 1e-12 * pre):
            failed.append("energy")
        rr_direct = float(res.r @ res.r)
        if abs(rr_direct - res.rr) > 1e-12 * res.yy:
            failed.append("norm_consistency")
    if res.reason != oracle.CONVERGED or not res.rr <= p.eps ** 2 * res.yy:
        failed.append("converged")
    # 4. stop counts: cap binds exactly, eps between tails fixes the count
    res = oracle.solve(psi, y, 0.0, 2, lib=lib)
    if res.iters != 2 or res.reason != oracle.MAX_ITERS:
        failed.append("cap")
    res = oracle.solve(psi, y, 0.25, 20, lib=lib)
    if res.iters != 5:
        failed.append("eps_stop_count")
    # 5. the FP64-y entry: exact dyadic recovery with more than 24 bits
    x64 = np.zeros(16)
    x64[[1, 4, 9]] = [0.5 + 2.0 ** -30, -(0.25 + 2.0 ** -40), 0.125 + 2.0 ** -35]
    psi64h = psi.astype(np.float64)
    res = oracle.solve64(psi64h, psi64h @ x64, 0.0, 10, lib=lib)
    if res.idx.tolist() != [1, 4, 9] or not np.array_equal(res.x, x64) or res.rr != 0.0:
        failed.append("fp64_dyadic")
    # 6. replay on an orthonormal dictionary, support forced out of order: the
    #    coefficients are the x values and the deficits max_remaining |x| - |x_i|
    rng = np.random.default_rng(11)
    q = mpgen.qr_orthonormal_dictionary(rng, 24)
    xo = np.zeros(24)
    order = [17, 3, 9, 21, 0]
    xo[order] = [0.3, -1.7, 0.9, -0.2, 1.1]
    rep = oracle.replay(q, q @ xo, order, check_ties=True, y64=True, lib=lib)
    want = [max(abs(xo[j]) for j in order[t:]) - abs(xo[i]) for t, i in enumerate(order)]
    if (np.max(np.abs(rep.coef - xo[order])) > 1e-14
            or np.max(np.abs(rep.deficit - np.array(want))) > 1e-14):
        failed.append("replay_orthonormal")
    # 7. replaying the free run's own sequence gives the free run back
    res = oracle.solve(p.psi, p.y, p.eps, p.max_iters, lib=lib)
    for ties in (True, False):
        rep = oracle.replay(p.psi, p.y, res.idx, check_ties=ties, lib=lib)
        if not (np.array_equal(rep.x, res.x) and np.array_equal(rep.r, res.r)):
            failed.append("replay_own_sequence")
            break
    return failed


def test_unmodified_oracle_passes_battery():
    assert _pin_battery(oracle._load()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(tmp_path, name):
    lib = _build_variant(tmp_path, name, MUTANTS[name])
    failed = _pin_battery(lib)
    assert failed, f"mutant {name} passed every pin"
