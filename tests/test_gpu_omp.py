"""GPU parity of Orthogonal Matching Pursuit (mp_solve_omp) against the FP64
OMP oracle (oracle.omp), through the C ABI.

Index sequences must agree step for step until a difference the oracle's
top-two gap allows (gap <= 1e-5 ||r|| + 2 ||r_gpu - r_ora|| + 2 e32 at that
step, the bound of the MP parity protocol); at that step the GPU's x~ and r
(a re-run capped there) are compared with the oracle's least-squares fit
(x~ relative to ||x~||, r relative to ||y||, 1e-5).  Every step of the GPU
run is checked on its own state (P-local: the atom is the FP64 argmax of
|Psi^T r_t| wherever the top-two gap exceeds 1e-5 ||r_t||), its final x~ and
r against the least-squares fit on its own atoms (an OMP state depends only
on the set of atoms), and its end state must be an OMP state: r orthogonal
to the selected atoms, y = Psi x~ + r and the stopping rule.
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
from oracle import omp as omp_oracle
from parity import fp32_dot_bound
from wholerun import local_checks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()


def _cm(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32).T)).cuda().t()


def _decoder(psi):
    from paper_0809_1833_amd.mp import Decoder
    return Decoder(_cm(psi))


def _gpu(dec, y, eps, T, cap=None, trace_r=False):
    yd = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()
    cap = T if cap is None else cap
    out = dec.solve(yd, eps, T, trace_cap=min(cap, dec.n) if cap else 0, omp=True,
                    trace_r=trace_r and cap > 0)
    torch.cuda.synchronize()
    g = dict(x=out["x"].cpu().numpy(), r=out["r"].cpu().numpy(), iters=out["iters"],
             stop=out["stop"], rr=out["rr"])
    if cap:
        g.update(idx=out["idx"].cpu().numpy(), coef=out["coef"].cpu().numpy(),
                 rr_trace=out["rr_trace"].cpu().numpy())
        if trace_r:
            g.update(r_trace=out["r_trace"].cpu().numpy())
    return g


def _check_end_state(psi, y, g, eps):
    y64 = y.astype(np.float64)
    yn = float(np.linalg.norm(y64))
    sel = g["idx"][:g["iters"]]
    ps = np.asarray(psi, dtype=np.float64)[:, sel]
    r = g["r"].astype(np.float64)
    assert np.max(np.abs(ps.T @ r)) <= TOL * yn, "r not orthogonal to the selected atoms"
    nz = np.flatnonzero(g["x"])
    assert set(nz.tolist()) <= set(sel.tolist()), "x~ nonzero off the selected atoms"
    defect = y64 - ps @ g["x"][sel].astype(np.float64) - r
    assert np.linalg.norm(defect) <= TOL * yn, "y != Psi x~ + r"
    if g["stop"] == "converged":
        assert float(r @ r) <= (eps * yn) ** 2 * (1 + 1e-5)


def _errs(gx, gr, ox, orr, yn):
    xe = np.linalg.norm(gx.astype(np.float64) - ox) / max(np.linalg.norm(ox), 1e-300)
    re = np.linalg.norm(gr.astype(np.float64) - orr) / max(yn, 1e-300)
    return float(xe), float(re)


def _ls_state(psi, y, sel):
    """The OMP state on the atoms `sel`: the least-squares fit of y (the
    oracle's own fit, FP64) and its residual."""
    y64 = np.asarray(np.asarray(y, dtype=np.float32), dtype=np.float64)
    x = np.zeros(psi.shape[1])
    if len(sel) == 0:
        return x, y64
    ps = np.asarray(psi, dtype=np.float64)[:, sel]
    xs = omp_oracle._fit(ps, y64)
    x[sel] = xs
    return x, omp_oracle._residual(y64, ps, xs)


def _parity(psi, y, eps, T, dec, oracle_cap=None):
    cap = T if oracle_cap is None else min(T, oracle_cap)
    ora = omp_oracle.solve_omp(psi, y, eps, cap)
    g = _gpu(dec, y, eps, T, trace_r=True)
    L = min(g["iters"], ora.iters)
    diff = np.flatnonzero(g["idx"][:L] != ora.idx[:L])
    t_star = int(diff[0]) if diff.size else L
    n = psi.shape[0]
    yn = float(np.linalg.norm(y.astype(np.float64)))
    full = t_star == L and g["iters"] == ora.iters and oracle_cap is None
    if full:
        assert omp_oracle.REASONS[ora.reason] == g["stop"]
        xe, re = _errs(g["x"], g["r"], ora.x, ora.r, yn)
        assert xe <= TOL and re <= TOL, (xe, re)
    elif t_star > 0:
        # the state at the end of the common prefix: the GPU run capped there,
        # the oracle's fit on the same atoms
        gp = _gpu(dec, y, 0.0, t_star, cap=0)
        ox, orr = _ls_state(psi, y, ora.idx[:t_star])
        xe, re = _errs(gp["x"], gp["r"], ox, orr, yn)
        assert xe <= TOL and re <= TOL, (t_star, xe, re)
        if t_star < L:
            # a difference at t* must be one the oracle's top-two gap allows
            rn = float(np.linalg.norm(orr))
            dr = float(np.linalg.norm(gp["r"].astype(np.float64) - orr))
            allowed = 1e-5 * rn + 2 * dr + 2 * fp32_dot_bound(n, rn)
            assert ora.gap[t_star] <= allowed, (t_star, ora.gap[t_star], allowed)
    # every step of the GPU run on its own state, and its end state against
    # the least-squares fit on its own atoms
    w = local_checks(psi, y, g)
    assert w.misses == 0
    ox, orr = _ls_state(psi, y, g["idx"][:g["iters"]])
    xe, re = _errs(g["x"], g["r"], ox, orr, yn)
    assert xe <= TOL and re <= TOL, ("end", xe, re)
    _check_end_state(psi, y, g, eps)
    return t_star, ora, g


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parity_small_workload(seed):
    p = mpgen.make_problem("c0", seed)
    print(f"[omp c0 seed={seed}]", flush=True)
    with _decoder(p.psi) as dec:
        t_star, ora, g = _parity(p.psi, p.y, p.eps, p.max_iters, dec)
    assert t_star == ora.iters == g["iters"]


def test_parity_2048x8192():
    p = mpgen.make_problem("c1a", 0)
    print("[omp c1a seed=0]", flush=True)
    with _decoder(p.psi) as dec:
        t_star, ora, g = _parity(p.psi, p.y, p.eps, p.max_iters, dec)
    print(t_star, ora.iters, g["iters"], flush=True)
    assert t_star >= min(ora.iters, 100)


def test_parity_8192x32768_whole_run():
    """The OMP decode the benchmark times: the oracle's free run for 48 steps
    (x~ and r compared there), then every step of the GPU run."""
    p = mpgen.make_problem("c1b", 0)
    print("[omp c1b seed=0]", flush=True)
    with _decoder(p.psi) as dec:
        t_star, ora, g = _parity(p.psi, p.y, p.eps, p.max_iters, dec, oracle_cap=48)
    assert t_star == 48
    assert g["stop"] == "converged"


def test_hadamard_exact_and_ties():
    """Orthonormal Hadamard columns (entries +-1/16) and dyadic nonzeros: every
    step is exact in FP32 (OMP is MP here), so indices (equal |c| -> smallest
    index first) and x~ are bit-exact."""
    n = 256
    psi = mpgen.hadamard_dictionary(n)
    x = np.zeros(n, dtype=np.float32)
    x[[7, 30, 31, 100, 200]] = [0.5, -0.5, 0.25, 0.5, -0.125]
    y = mpgen.encode(psi, x)
    with _decoder(psi) as dec:
        g = _gpu(dec, y, 0.0, 20)
    assert g["idx"].tolist() == [7, 30, 100, 31, 200]
    assert np.array_equal(g["x"], x) and not np.any(g["r"])


def test_recovers_sparse_signal():
    rng = np.random.default_rng(12)
    psi = mpgen.gaussian_unit_dictionary(rng, 128, 512)
    x, sup = mpgen.sparse_signal(rng, rng, 512, 8)
    y = mpgen.encode(psi, x, sup)
    with _decoder(psi) as dec:
        g = _gpu(dec, y, 1e-6, 100)
    assert g["iters"] == 8 and g["stop"] == "converged"
    assert sorted(g["idx"].tolist()) == sup.tolist()
    assert np.linalg.norm(g["x"] - x) <= 1e-5 * np.linalg.norm(x)


@pytest.mark.parametrize("n,m", [(1, 1), (3, 5), (70, 9), (250, 1000), (520, 300), (4096, 2049)])
def test_ragged_and_extreme_shapes(n, m):
    rng = np.random.default_rng(n * 31 + m)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    k = max(1, min(m // 8, n // 4, 6))
    x, sup = mpgen.sparse_signal(rng, rng, m, k)
    y = mpgen.encode(psi, x, sup)
    print(f"[omp shape {n}x{m}]", flush=True)
    with _decoder(psi) as dec:
        t_star, ora, g = _parity(psi, y, 1e-6, 300, dec)
    assert t_star >= min(ora.iters, 5)


def test_stop_rules_and_edges():
    p = mpgen.make_problem("c0", 3)
    with _decoder(p.psi) as dec:
        g = _gpu(dec, p.y, 1e-6, 0)
        assert g["iters"] == 0 and g["stop"] == "max_iters"
        g = _gpu(dec, p.y, 1e-6, 3)
        assert g["iters"] == 3 and g["stop"] == "max_iters"
        ora = omp_oracle.solve_omp(p.psi, p.y, 1e-6, 3)
        assert g["idx"].tolist() == ora.idx.tolist()
        g = _gpu(dec, p.y, 2.0, 10)
        assert g["iters"] == 0 and g["stop"] == "converged"
        g = _gpu(dec, np.zeros(p.n, np.float32), 1e-6, 10)
        assert g["iters"] == 0 and g["stop"] == "zero_input" and not np.any(g["x"])
    # at most N atoms: with eps = 0 the run ends by the cap N, or stalls once
    # r is at the FP32 floor
    rng = np.random.default_rng(5)
    psi = mpgen.gaussian_unit_dictionary(rng, 16, 64)
    y = mpgen.encode(psi, *mpgen.sparse_signal(rng, rng, 64, 12))
    with _decoder(psi) as dec:
        g = _gpu(dec, y, 0.0, 1000)
    assert g["iters"] <= 16 and g["stop"] in ("max_iters", "stalled", "converged")
    _check_end_state(psi, y, g, 0.0)


def test_duplicate_atom_is_not_refitted():
    """Two identical atoms: the second can only come up once r is orthogonal
    to the first, and then it adds nothing; the run must not break down."""
    rng = np.random.default_rng(8)
    psi = np.array(mpgen.gaussian_unit_dictionary(rng, 32, 40))
    psi[:, 5] = psi[:, 2]
    psi = np.asfortranarray(psi)
    x = np.zeros(40, np.float32)
    x[[2, 9, 20]] = [1.0, -0.7, 0.4]
    y = mpgen.encode(psi, x)
    with _decoder(psi) as dec:
        g = _gpu(dec, y, 0.0, 40)
    assert g["stop"] in ("stalled", "max_iters", "converged")
    assert not (2 in g["idx"][:g["iters"]] and 5 in g["idx"][:g["iters"]])
    _check_end_state(psi, y, g, 0.0)


def test_determinism_and_rejects():
    from paper_0809_1833_amd import mp
    p = mpgen.make_problem("c0", 6)
    with _decoder(p.psi) as dec:
        a = _gpu(dec, p.y, p.eps, p.max_iters)
        b = _gpu(dec, p.y, p.eps, p.max_iters)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["idx"], b["idx"])
    from paper_0809_1833_amd.mp import Decoder
    with Decoder(_cm(p.psi), storage="bf16") as d16:
        opts = mp.Opts(1e-5, 10, 0, 0)
        x = torch.empty(p.m, device="cuda")
        y = torch.from_numpy(p.y).cuda()
        with pytest.raises(mp.MPError) as e:
            mp.mp_solve_omp(d16.handle, y.data_ptr(), x.data_ptr(), None, opts)
        assert e.value.status == mp.MP_EINVAL
