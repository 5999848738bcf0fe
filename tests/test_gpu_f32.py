"""GPU parity of the FP32 single-signal decoder (mp_solve) against the FP64 oracle.

All calls go through the C ABI (libmp.so via its ctypes binding).  Inputs are
the seeded workloads of ``mpgen``; expected values come from the oracle only.
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from parity import run_parity
from wholerun import whole_run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(psi: np.ndarray):
    """(N, M) column-major numpy -> (N, M) column-major CUDA tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(psi, dtype=np.float32).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _decoder(psi, storage="f32", check_norms=True):
    from paper_0809_1833_amd.mp import Decoder
    return Decoder(_dev(psi), storage=storage, check_norms=check_norms)


def _gpu_solver(dec, y):
    yd = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()

    def solve(eps, max_iters, cap):
        out = dec.solve(yd, eps, max_iters, trace_cap=cap)
        torch.cuda.synchronize()
        res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                   rr=out["rr"], yy=out["yy"])
        if cap:
            res.update(idx=_np(out["idx"]), coef=_np(out["coef"]), rr_trace=_np(out["rr_trace"]))
        else:
            res.update(idx=np.zeros(0, np.int32), coef=np.zeros(0, np.float32),
                       rr_trace=np.zeros(0))
        return res
    return solve


def _gpu_traced(dec, y, eps, max_iters, **kw):
    """One decode with the full trace, residuals included, as numpy arrays."""
    yd = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()
    out = dec.solve(yd, eps, max_iters, trace_cap=max(max_iters, 1), trace_r=True, **kw)
    torch.cuda.synchronize()
    return dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                idx=_np(out["idx"]), coef=_np(out["coef"]), r_trace=_np(out["r_trace"]))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()  # fail loudly if the HIP library is not built


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parity_small_workload(seed):
    """N=256, M=1024, K=10, eps=1e-6, T=2000 (several tiles)."""
    p = mpgen.make_problem("c0", seed)
    print(f"[c0 seed={seed}]", flush=True)
    with _decoder(p.psi) as dec:
        rep = run_parity(p.psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y))
    assert rep.full_match, rep


@pytest.mark.parametrize("seed", [0, 1])
def test_parity_2048x8192(seed):
    """N=2048, M=8192, K=128, eps=1e-5, T=20K: full oracle run, then every
    step of the GPU run checked (P-local, P-replay, the final x~ and r)."""
    p = mpgen.make_problem("c1a", seed)
    print(f"[c1a seed={seed}]", flush=True)
    with _decoder(p.psi) as dec:
        rep = run_parity(p.psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y))
        print(rep, flush=True)
        assert rep.prefix >= min(rep.iters_ora, 100)
        w = whole_run(p.psi, p.y, p.eps, _gpu_traced(dec, p.y, p.eps, p.max_iters))
    print(w, flush=True)


def test_parity_8192x32768_whole_run():
    """N=8192, M=32768 (1 GiB dictionary), the benchmarked decode: the oracle's
    free run to its end (index prefix, legitimacy of the first difference),
    then every one of the GPU's steps correlated in FP64 (the selection is the
    FP64 argmax wherever the top-two gap exceeds 1e-5 ||r||, the coefficient
    within the FP32 bound), the oracle's replay of the GPU's atoms (each a
    near tie of the oracle's own state; x~ and r at the end within 1e-5)."""
    p = mpgen.make_problem("c1b", 0)
    print("[c1b seed=0]", flush=True)
    with _decoder(p.psi) as dec:
        rep = run_parity(p.psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y), samples_after=3)
        print(rep, flush=True)
        assert rep.prefix >= 48
        g = _gpu_traced(dec, p.y, p.eps, p.max_iters)
    print(f"[c1b whole run: {g['iters']} steps]", flush=True)
    w = whole_run(p.psi, p.y, p.eps, g)
    print(w, flush=True)
    assert w.steps == rep.iters_gpu and w.exact_steps > 0.9 * w.steps


@pytest.mark.parametrize("n,m", [(250, 1000), (1, 1), (3, 5), (64, 4), (100, 7), (520, 300),
                                 (16384, 64), (4096, 2049), (4160, 3001), (4100, 700),
                                 (16384, 16384)])
def test_ragged_and_extreme_shapes(n, m):
    """Column lengths that are not multiples of the tile, tiny and maximum N
    (at M = 16384 with the balanced column shares active); N = 4160 and 4100
    (padded to 4160) end each column in a ragged block after two full ones."""
    rng = np.random.default_rng(n * 7919 + m)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    k = max(1, min(m // 8, n // 4, 6))
    x, sup = mpgen.sparse_signal(rng, rng, m, k)
    y = mpgen.encode(psi, x, sup)
    print(f"[shape {n}x{m}]", flush=True)
    with _decoder(psi) as dec:
        rep = run_parity(psi, y, 1e-6, 300, _gpu_solver(dec, y))
    assert rep.prefix >= min(rep.iters_ora, 20)


def test_leading_dimension_larger_than_n():
    p = mpgen.make_problem("c0", 5)
    big = np.zeros((p.n + 13, p.m), dtype=np.float32, order="F")
    big[: p.n] = p.psi
    from paper_0809_1833_amd.mp import Decoder
    t = torch.from_numpy(np.ascontiguousarray(big.T)).cuda().t()[: p.n]
    assert t.stride() == (1, p.n + 13)
    with Decoder(t) as dec:
        rep = run_parity(p.psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y))
    assert rep.full_match


def test_hadamard_ties_exact():
    """Equal |c| -> smallest index (eq. 16), bit-exact on the GPU."""
    psi = mpgen.hadamard_dictionary(16)
    x = np.zeros(16, np.float32)
    x[[3, 7, 11, 12, 14, 15]] = [-0.5, 0.5, 0.5, 0.25, -0.25, 0.125]
    y = mpgen.encode(psi, x)
    with _decoder(psi) as dec:
        g = _gpu_solver(dec, y)(0.0, 20, 20)
    assert g["idx"].tolist() == [3, 7, 11, 12, 14, 15]
    assert g["coef"].tolist() == [-0.5, 0.5, 0.5, 0.25, -0.25, 0.125]
    assert np.array_equal(g["x"], x) and g["iters"] == 6 and g["stop"] == "converged"


def test_hadamard_large_orthonormal():
    n = 4096
    psi = mpgen.hadamard_dictionary(n)
    rng = np.random.default_rng(3)
    sup = np.sort(rng.choice(n, size=40, replace=False))
    x = np.zeros(n, np.float32)
    x[sup] = rng.integers(1, 2 ** 10, size=40) * np.where(rng.random(40) < .5, -1, 1) / 2 ** 10
    y = mpgen.encode(psi, x)
    with _decoder(psi) as dec:
        g = _gpu_solver(dec, y)(1e-7, 100, 100)
    ora = oracle.solve(psi, y, 1e-7, 100)
    assert g["idx"].tolist() == ora.idx.tolist()
    assert g["iters"] == 40
    np.testing.assert_allclose(g["x"], x, rtol=0, atol=1e-6)


def test_stop_rules():
    p = mpgen.make_problem("c0", 0)
    with _decoder(p.psi) as dec:
        s = _gpu_solver(dec, p.y)
        assert s(p.eps, 0, 0)["iters"] == 0 and s(p.eps, 0, 0)["stop"] == "max_iters"
        r = s(1.0, 10, 10)
        assert r["iters"] == 0 and r["stop"] == "converged"
        r = s(p.eps, 7, 10)
        assert r["iters"] == 7 and r["stop"] == "max_iters"
        z = _gpu_solver(dec, np.zeros(p.n, np.float32))(p.eps, 10, 10)
        assert z["iters"] == 0 and z["stop"] == "zero_input" and not z["x"].any()
        assert np.array_equal(s(0.0, 0, 0)["r"], p.y)


def test_stalled():
    psi = np.asfortranarray(np.array([[1.0, 1.0, -1.0], [0.0, 0.0, 0.0]], dtype=np.float32))
    with _decoder(psi) as dec:
        g = _gpu_solver(dec, np.array([0.0, 1.0], np.float32))(0.0, 5, 5)
    assert g["iters"] == 0 and g["stop"] == "stalled"


def test_determinism():
    """Identical inputs give bit-identical traces (fixed reduction order)."""
    p = mpgen.make_problem("c1a", 2)
    with _decoder(p.psi) as dec:
        s = _gpu_solver(dec, p.y)
        a = s(p.eps, 300, 300)
        b = s(p.eps, 300, 300)
    assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(a["coef"], b["coef"])
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["r"], b["r"])


def test_error_paths():
    from paper_0809_1833_amd import mp
    p = mpgen.make_problem("c0", 0)
    bad = np.array(p.psi, order="F")
    bad[:, 17] *= 1.01
    with pytest.raises(mp.MPError) as e:
        _decoder(bad)
    assert e.value.status == mp.MP_ENOTNORM and "column 17" in str(e.value)
    _decoder(bad, check_norms=False).close()
    bad[3, 40] = np.nan
    with pytest.raises(mp.MPError) as e:
        _decoder(bad, check_norms=False)
    assert e.value.status == mp.MP_ENONFINITE
    with _decoder(p.psi) as dec:
        yd = torch.from_numpy(p.y).cuda()
        with pytest.raises(mp.MPError) as e:
            dec.solve(yd, -1.0, 10)
        assert e.value.status == mp.MP_EINVAL
        with pytest.raises(mp.MPError) as e:
            dec.solve(yd, 1e-5, -3)
        assert e.value.status == mp.MP_EINVAL
        ynan = yd.clone()
        ynan[5] = float("inf")
        with pytest.raises(mp.MPError) as e:
            dec.solve(ynan, 1e-5, 10)
        assert e.value.status == mp.MP_ENONFINITE
        # the context is still usable after errors
        out = dec.solve(yd, p.eps, p.max_iters)
        assert out["stop"] == "converged"


def test_storage_copy_is_exact():
    p = mpgen.make_problem("c0", 0)
    with _decoder(p.psi) as dec:
        codes, scales = dec.storage_copy()
        assert scales is None
        assert np.array_equal(_np(codes), p.psi)


def test_profiling_counts_real_launches():
    """Kernel timing counts the launches that ran a correlation pass: all of
    them with windows of one launch, whole windows only with longer ones
    (windows are cut from the start of each chunk of launches, whose lengths
    follow the residual's decay); the one-launch form counts its steps."""
    p = mpgen.make_problem("c0", 0)
    y = torch.from_numpy(p.y).cuda()
    with _decoder(p.psi) as dec:
        dec.set_profiling(1)
        out = dec.solve(y, p.eps, p.max_iters, step_launches=True)
        ms, n = dec.kernel_time()
        assert n == out["iters"] and ms > 0
        dec.set_profiling(4)
        out = dec.solve(y, p.eps, p.max_iters, step_launches=True)
        ms, n = dec.kernel_time()
        assert n % 4 == 0 and 0 < n <= out["iters"] and ms > 0
        out = dec.solve(y, p.eps, p.max_iters)  # one launch for the whole decode
        ms, n = dec.kernel_time()
        assert out["persistent"] and n == out["iters"] and ms > 0
        dec.set_profiling(0)
        dec.solve(y, p.eps, p.max_iters)
        assert dec.kernel_time()[1] == 0


@pytest.mark.parametrize("n,m", [(256, 1024), (250, 1000), (3, 5), (4100, 700)])
def test_residual_trace(n, m):
    """The residual trace holds each step's r bit for bit (rows below N only,
    including N not a multiple of four) and does not change the decode."""
    rng = np.random.default_rng(n + 31 * m)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    x, sup = mpgen.sparse_signal(rng, rng, m, max(1, min(m // 8, n // 4, 6)))
    y = mpgen.encode(psi, x, sup)
    with _decoder(psi) as dec:
        g = _gpu_traced(dec, y, 1e-6, 60)
        plain = _gpu_solver(dec, y)(1e-6, 60, 60)
        assert np.array_equal(g["idx"], plain["idx"]) and np.array_equal(g["x"], plain["x"])
        assert np.array_equal(g["r"], plain["r"])
        T = g["iters"]
        assert T > 0 and np.array_equal(g["r_trace"][T - 1], g["r"])
        for t in sorted({0, T // 2, T - 1}):
            part = _gpu_solver(dec, y)(0.0, t + 1, 0)
            assert np.array_equal(g["r_trace"][t], part["r"]), t
    with pytest.raises(Exception):
        from paper_0809_1833_amd import mp
        with _decoder(psi) as dec:
            yd = torch.from_numpy(y).cuda()
            tr = torch.zeros((4, n), device="cuda")
            t = mp.Trace(None, None, None, 4, tr.data_ptr(), n - 1)
            mp.mp_solve(dec.handle, yd.data_ptr(), torch.empty(m, device="cuda").data_ptr(),
                        None, mp.Opts(1e-6, 4, 0, 0), t)
