"""GPU parity of the FP64 single-signal decoder (mp_create_f64 / mp_solve_f64)
against the FP64 oracle on the same FP64 inputs.

Both sides compute in FP64; they differ only in the order of the additions
inside each inner product, so index sequences must agree step for step except
at ties within FP64 rounding, and x~ and r within 1e-12.  All calls go through
the C ABI; expected values come from the oracle (or are exact by
construction).
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from parity import U64, run_parity
from wholerun import whole_run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12       # x~ relative to ||x~||, r relative to ||y||
TOL_SEL = 1e-10   # a top-two gap above this fraction of ||r|| must be resolved exactly


def _dev(a: np.ndarray):
    """(N, M) column-major numpy FP64 -> (N, M) column-major CUDA tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _decoder(psi, check_norms=True):
    from paper_0809_1833_amd.mp import Decoder
    return Decoder(_dev(psi), storage="f64", check_norms=check_norms)


def _gpu_solver(dec, y):
    yd = torch.from_numpy(np.asarray(y, dtype=np.float64)).cuda()

    def solve(eps, max_iters, cap):
        out = dec.solve(yd, eps, max_iters, trace_cap=cap)
        torch.cuda.synchronize()
        res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                   rr=out["rr"], yy=out["yy"])
        if cap:
            res.update(idx=_np(out["idx"]), coef=_np(out["coef"]), rr_trace=_np(out["rr_trace"]))
        else:
            res.update(idx=np.zeros(0, np.int32), coef=np.zeros(0), rr_trace=np.zeros(0))
        return res
    return solve


def _parity(psi, y, eps, max_iters, dec, **kw):
    return run_parity(psi, y, eps, max_iters, _gpu_solver(dec, y), tol=TOL, tol_sel=TOL_SEL,
                      unit=U64, solver=oracle.solve64, **kw)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()  # fail loudly if the HIP library is not built


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parity_small_workload(seed):
    """N=256, M=1024, K=10, eps=1e-6 in FP64: the whole run matches."""
    p = mpgen.make_problem("c0", seed, precision="f64")
    print(f"[f64 c0 seed={seed}]", flush=True)
    with _decoder(p.psi) as dec:
        rep = _parity(p.psi, p.y, p.eps, p.max_iters, dec)
    assert rep.full_match, rep


def test_parity_2048x8192():
    """N=2048, M=8192, K=128, eps=1e-5, T=20K in FP64: full oracle run."""
    p = mpgen.make_problem("c1a", 0, precision="f64")
    print("[f64 c1a seed=0]", flush=True)
    with _decoder(p.psi) as dec:
        rep = _parity(p.psi, p.y, p.eps, p.max_iters, dec)
    print(rep, flush=True)
    assert rep.prefix >= min(rep.iters_ora, 200)


def test_parity_8192x32768_whole_run():
    """N=8192, M=32768 (2 GiB FP64 dictionary) at the full size: oracle prefix
    of 32 steps, then every step of the GPU run against FP64 correlations of
    its state (the exact argmax wherever the top-two gap exceeds 1e-10 ||r||)
    and the oracle's replay of its atoms (x~ and r at the end within
    1e-12)."""
    p = mpgen.make_problem("c1b", 0, precision="f64")
    print("[f64 c1b seed=0]", flush=True)
    with _decoder(p.psi) as dec:
        rep = _parity(p.psi, p.y, p.eps, p.max_iters, dec, oracle_cap=32, samples_after=2)
        print(rep, flush=True)
        assert rep.prefix == 32
        yd = torch.from_numpy(np.asarray(p.y, dtype=np.float64)).cuda()
        out = dec.solve(yd, p.eps, p.max_iters, trace_cap=p.max_iters, trace_r=True)
        torch.cuda.synchronize()
        g = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                 idx=_np(out["idx"]), coef=_np(out["coef"]), r_trace=_np(out["r_trace"]))
        del out
    print(f"[f64 c1b whole run: {g['iters']} steps]", flush=True)
    w = whole_run(p.psi, p.y, p.eps, g, tol=TOL, tol_sel=TOL_SEL, unit=U64, y64=True)
    print(w, flush=True)
    assert w.misses == 0 and w.exact_steps > 0.9 * w.steps


@pytest.mark.parametrize("n,m", [(250, 1000), (1, 1), (3, 5), (64, 4), (100, 7), (520, 300),
                                 (16384, 64), (4096, 2049), (16384, 16384)])
def test_ragged_and_extreme_shapes(n, m):
    """Column lengths that are not multiples of the tile, tiny and maximum N
    (a 128 KB FP64 residual in LDS; at M = 16384 beside the balanced
    shares' timing table)."""
    rng = np.random.default_rng(n * 7919 + m + 1)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m, dtype=np.float64)
    k = max(1, min(m // 8, n // 4, 6))
    x, sup = mpgen.sparse_signal(rng, rng, m, k, dtype=np.float64)
    y = mpgen.encode(psi, x, sup, dtype=np.float64)
    print(f"[f64 shape {n}x{m}]", flush=True)
    with _decoder(psi) as dec:
        rep = _parity(psi, y, 1e-9, 300, dec)
    assert rep.prefix >= min(rep.iters_ora, 20)


def test_orthonormal_recovery():
    """N = M orthonormal FP64 dictionary: MP is the sort of |x| (textbook
    reduction), K steps, x~ = x to FP64 rounding."""
    n, k = 256, 12
    rng = np.random.default_rng(11)
    q = mpgen.qr_orthonormal_dictionary(rng, n)
    sup = np.sort(rng.choice(n, size=k, replace=False))
    x = np.zeros(n)
    x[sup] = rng.standard_normal(k)
    y = q @ x
    with _decoder(q) as dec:
        g = _gpu_solver(dec, y)(1e-12, 100, 100)
    order = sup[np.argsort(-np.abs(q.T @ y)[sup], kind="stable")]
    assert g["iters"] == k and g["stop"] == "converged"
    assert g["idx"].tolist() == order.tolist()
    assert np.linalg.norm(g["x"] - x) <= 1e-13 * np.linalg.norm(x)


def test_dyadic_hadamard_bit_exact():
    """Hadamard columns (+-1/16) and dyadic nonzeros needing more than 24
    significant bits, with exact ties: every operation is exact in FP64, so
    the GPU must return the exact x~, r = 0 and the smallest index among equal
    |c| first (eq. 16)."""
    n = 256
    psi = mpgen.hadamard_dictionary(n).astype(np.float64)
    x = np.zeros(n)
    x[[3, 40, 77, 200, 201]] = [0.5 + 2.0 ** -30, 0.5 + 2.0 ** -30, -(0.25 + 2.0 ** -41),
                                0.125 + 2.0 ** -33, -(0.5 + 2.0 ** -30)]
    y = psi @ x
    ora = oracle.solve64(psi, y, 0.0, 20)
    with _decoder(psi) as dec:
        g = _gpu_solver(dec, y)(0.0, 20, 20)
    # |c| = 0.5 + 2^-30 three times (taken in index order), then 0.25 + 2^-41,
    # then 0.125 + 2^-33
    expect = [3, 40, 201, 77, 200]
    assert ora.idx.tolist() == expect
    assert g["idx"].tolist() == expect
    assert np.array_equal(g["x"], x) and not np.any(g["r"]) and g["rr"] == 0.0
    assert np.array_equal(g["coef"], ora.coef)


def test_stop_rules_and_edges():
    p = mpgen.make_problem("c0", 4, precision="f64")
    with _decoder(p.psi) as dec:
        solve = _gpu_solver(dec, p.y)
        ora = oracle.solve64(p.psi, p.y, 1e-3, 50)
        g = solve(1e-3, 50, 50)
        assert g["iters"] == ora.iters and g["stop"] == "converged"
        assert g["idx"].tolist() == ora.idx.tolist()
        g = solve(1e-9, 0, 0)
        assert g["iters"] == 0 and g["stop"] == "max_iters"
        g = solve(2.0, 10, 0)
        assert g["iters"] == 0 and g["stop"] == "converged"
        g = solve(1e-9, 3, 3)
        assert g["iters"] == 3 and g["stop"] == "max_iters"
        zero = _gpu_solver(dec, np.zeros(p.n))(1e-6, 10, 0)
        assert zero["iters"] == 0 and zero["stop"] == "zero_input"
        assert not np.any(zero["x"])


def test_determinism():
    p = mpgen.make_problem("c0", 6, precision="f64")
    with _decoder(p.psi) as dec:
        a = _gpu_solver(dec, p.y)(p.eps, p.max_iters, 64)
        b = _gpu_solver(dec, p.y)(p.eps, p.max_iters, 64)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["r"], b["r"])
    assert np.array_equal(a["idx"], b["idx"])


def test_rejects():
    from paper_0809_1833_amd import mp
    p = mpgen.make_problem("c0", 0, precision="f64")
    bad = np.array(p.psi)
    bad[:, 5] *= 1.01
    with pytest.raises(mp.MPError) as e:
        _decoder(bad)
    assert e.value.status == mp.MP_ENOTNORM
    bad[:, 5] = np.nan
    with pytest.raises(mp.MPError) as e:
        _decoder(bad, check_norms=False)
    assert e.value.status == mp.MP_ENONFINITE
    with _decoder(p.psi) as dec:
        y = torch.from_numpy(p.y).cuda()
        y[3] = float("inf")
        with pytest.raises(mp.MPError) as e:
            dec.solve(y, 1e-6, 10)
        assert e.value.status == mp.MP_ENONFINITE
        opts = mp.Opts(1e-5, 10, 0, 0)
        x32 = torch.empty(p.m, device="cuda")
        y32 = torch.zeros(p.n, device="cuda")
        with pytest.raises(mp.MPError) as e:   # an FP64 context through the FP32 entry
            mp.mp_solve(dec.handle, y32.data_ptr(), x32.data_ptr(), None, opts)
        assert e.value.status == mp.MP_EINVAL
    p32 = mpgen.make_problem("c0", 0)
    from paper_0809_1833_amd.mp import Decoder
    with Decoder(torch.from_numpy(np.ascontiguousarray(p32.psi.T)).cuda().t()) as d32:
        opts = mp.Opts(1e-5, 10, 0, 0)
        x64 = torch.empty(p.m, dtype=torch.float64, device="cuda")
        y64 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        with pytest.raises(mp.MPError) as e:   # an FP32 context through the FP64 entry
            mp.mp_solve_f64(d32.handle, y64.data_ptr(), x64.data_ptr(), None, opts)
        assert e.value.status == mp.MP_EINVAL


def test_storage_copy_roundtrip():
    p = mpgen.make_problem("c0", 2, precision="f64")
    with _decoder(p.psi) as dec:
        codes, scales = dec.storage_copy()
        torch.cuda.synchronize()
    assert scales is None
    assert np.array_equal(_np(codes), p.psi)
