"""GPU parity of the sign-bit Bernoulli decoder (mp_create_signs + mp_solve)
against the FP64 oracle on the dictionary the bits stand for (eq. 13).

All calls go through the C ABI.  Inputs come from ``mpgen``'s sign-bit
problems; expected values come from the oracle only (``oracle.signs`` reads
the bits back into +-1/sqrt(N) FP64 entries and runs the FP64 MP)."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from oracle import signs as osigns
from parity import run_parity
from wholerun import whole_run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()


def _np(t):
    return t.detach().cpu().numpy()


def _decoder(bits, n):
    from paper_0809_1833_amd.mp import Decoder
    dev = torch.from_numpy(np.ascontiguousarray(bits).view(np.int32)).cuda()
    return Decoder(dev, storage="sign", n=n)


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


def _sylvester(n):
    h = np.array([[1]], dtype=np.int8)
    while h.shape[0] < n:
        h = np.kron(np.array([[1, 1], [1, -1]], dtype=np.int8), h)
    return h


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parity_small_workload(seed):
    """N=256, M=1024, K=10, eps=1e-6, T=2000 on a sign-bit dictionary."""
    p = mpgen.make_sign_problem("c0", seed)
    print(f"[sign c0 seed={seed}]", flush=True)
    psi = osigns.unpack(p.bits, p.n)
    with _decoder(p.bits, p.n) as dec:
        rep = run_parity(psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y))
    assert rep.full_match, rep


def test_parity_2048x8192():
    p = mpgen.make_sign_problem("c1a", 0)
    print("[sign c1a seed=0]", flush=True)
    psi = osigns.unpack(p.bits, p.n)
    with _decoder(p.bits, p.n) as dec:
        rep = run_parity(psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y))
    print(rep, flush=True)
    assert rep.prefix >= min(rep.iters_ora, 100)


def test_parity_8192x32768_whole_run():
    """The benchmark size (N=8192, M=32768, 32 MiB of bits), in the launch
    configuration the benchmark uses (the persistent decode): oracle prefix
    of 24 steps, then every step of the GPU run against FP64 correlations of
    its state (the exact argmax wherever the top-two gap exceeds 1e-5 ||r||),
    and the oracle's replay of its atoms (near ties of the oracle's states;
    x~ and r at the end within 1e-5)."""
    p = mpgen.make_sign_problem("c1b", 0)
    print("[sign c1b seed=0]", flush=True)
    psi = osigns.unpack(p.bits, p.n)
    with _decoder(p.bits, p.n) as dec:
        rep = run_parity(psi, p.y, p.eps, p.max_iters, _gpu_solver(dec, p.y), oracle_cap=24,
                         samples_after=2)
        print(rep, flush=True)
        assert rep.prefix == 24
        yd = torch.from_numpy(np.asarray(p.y, dtype=np.float32)).cuda()
        out = dec.solve(yd, p.eps, p.max_iters, trace_cap=p.max_iters, trace_r=True)
        torch.cuda.synchronize()
        assert out["persistent"]
        g = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                 idx=_np(out["idx"]), coef=_np(out["coef"]), r_trace=_np(out["r_trace"]))
        del out
    print(f"[sign c1b whole run: {g['iters']} steps]", flush=True)
    w = whole_run(psi, p.y, p.eps, g)
    print(w, flush=True)
    assert w.misses == 0 and w.exact_steps > 0.9 * w.steps


@pytest.mark.parametrize("n,m", [(1, 5), (3, 40), (33, 17), (100, 1000), (2047, 300),
                                 (2049, 300), (6000, 129), (8192, 70), (8193, 33),
                                 (12000, 100), (16384, 40)])
def test_parity_ragged_shapes(n, m):
    """Columns of one and two 16-byte chunks per lane (N <= 8192 and above),
    N not a multiple of 4, 32 or 64, M below and not a multiple of the
    workgroup's column count."""
    rng = np.random.default_rng(n * 7 + m)
    s = mpgen.bernoulli_signs(rng, n, m)
    k = max(1, min(6, n // 8, m // 4))
    x, sup = mpgen.sparse_signal(rng, rng, m, k)
    y = mpgen.encode_signs(s, x, sup)
    bits = mpgen.pack_signs(s, ldw=(n + 31) // 32 + 1)
    print(f"[sign shape {n}x{m}]", flush=True)
    psi = osigns.unpack(bits, n)
    with _decoder(bits, n) as dec:
        rep = run_parity(psi, y, 1e-6, 200, _gpu_solver(dec, y))
    assert rep.prefix >= min(rep.iters_ora, 5), rep


@pytest.mark.parametrize("n,m,planted", [(8192, 33000, [130, 855, 28940]),
                                         (8200, 16500, [70, 8075, 16479])])
def test_parity_many_columns(n, m, planted):
    """M above 256 workgroups' worth of columns: a workgroup scores at most
    128 columns (64 for N > 8192), so the decode takes more workgroups.  The
    largest atoms sit where a share of 144 (80) columns per workgroup would
    have left columns unscored."""
    rng = np.random.default_rng(n + m)
    s = mpgen.bernoulli_signs(rng, n, m)
    sup = np.sort(np.array(planted + [5, m // 2, m - 1], dtype=np.int64))
    x = np.zeros(m, np.float32)
    x[sup] = rng.standard_normal(sup.size).astype(np.float32) * 0.1
    x[planted] = np.array([4.0, -3.0, 2.5], np.float32)
    y = mpgen.encode_signs(s, x, sup)
    bits = mpgen.pack_signs(s)
    del s
    print(f"[sign many columns {n}x{m}]", flush=True)
    psi = osigns.unpack(bits, n)
    with _decoder(bits, n) as dec:
        out = _gpu_solver(dec, y)(1e-6, 40, 8)
        assert list(out["idx"][:3]) == planted, out["idx"][:8]
        rep = run_parity(psi, y, 1e-6, 40, _gpu_solver(dec, y))
    assert rep.prefix >= min(rep.iters_ora, 5), rep


@pytest.mark.parametrize("case", ["c0", "c1a", "c1b", "100x1000", "2047x300", "1x5",
                                  "12000x16384"])
def test_persistent_matches_step_launches(case):
    """Where the whole decode fits one persistent launch (every workgroup's
    share of the bits in LDS), it gives the stepping form's results bit for
    bit: x~, r, the iteration count and every step's index, coefficient and
    ||r||^2.  12000 x 16384 takes the two-chunks-per-lane variant (64
    columns of 94 chunks per workgroup, 96 KB of LDS)."""
    if case.startswith("c"):
        p = mpgen.make_sign_problem(case, 0)
        n, m, bits, y, eps, t_cap = p.n, p.m, p.bits, p.y, p.eps, p.max_iters
    else:
        n, m = (int(v) for v in case.split("x"))
        rng = np.random.default_rng(n * 31 + m)
        s = mpgen.bernoulli_signs(rng, n, m)
        k = max(1, min(6, n // 8, m // 4))
        x, sup = mpgen.sparse_signal(rng, rng, m, k)
        y = mpgen.encode_signs(s, x, sup)
        bits = mpgen.pack_signs(s)
        eps, t_cap = 1e-6, 200
    print(f"[sign persistent {case}]", flush=True)
    cap = int(min(t_cap, 4096))
    with _decoder(bits, n) as dec:
        yd = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()
        a = dec.solve(yd, eps, t_cap, trace_cap=cap, trace_r=n * cap <= 2 ** 26)
        b = dec.solve(yd, eps, t_cap, trace_cap=cap, step_launches=True,
                      trace_r=n * cap <= 2 ** 26)
        torch.cuda.synchronize()
    assert a["persistent"] and not b["persistent"]
    assert a["iters"] == b["iters"] and a["stop"] == b["stop"]
    assert a["rr"] == b["rr"]
    keys = ["x", "r", "idx", "coef", "rr_trace"] + (["r_trace"] if "r_trace" in a else [])
    for key in keys:
        assert np.array_equal(_np(a[key]), _np(b[key])), key
    if "r_trace" in a and a["iters"]:
        assert np.array_equal(_np(a["r_trace"][-1]), _np(a["r"]))


def test_persistent_wait_limit_fails_cleanly(monkeypatch):
    """The persistent decode's waits cut to two polls (MP_SIGN_SPIN_LIMIT=1,
    read by the library at each decode): over the decode's thousands of
    steps some wait gives up, the run is marked failed and every workgroup
    leaves through its own bounded wait, so the call returns MP_EDEVICE; the
    context then decodes as before, bit for bit with the stepping form."""
    from paper_0809_1833_amd import mp
    p = mpgen.make_sign_problem("c1a", 0)
    print("[sign persistent wait limit]", flush=True)
    with _decoder(p.bits, p.n) as dec:
        yd = torch.from_numpy(np.asarray(p.y, dtype=np.float32)).cuda()
        monkeypatch.setenv("MP_SIGN_SPIN_LIMIT", "1")
        with pytest.raises(mp.MPError) as e:
            dec.solve(yd, p.eps, p.max_iters)
        assert e.value.status == mp.MP_EDEVICE
        monkeypatch.delenv("MP_SIGN_SPIN_LIMIT")
        a = dec.solve(yd, p.eps, p.max_iters)
        b = dec.solve(yd, p.eps, p.max_iters, step_launches=True)
        torch.cuda.synchronize()
    assert a["persistent"] and a["iters"] == b["iters"] and a["stop"] == b["stop"]
    assert np.array_equal(_np(a["x"]), _np(b["x"])) and np.array_equal(_np(a["r"]), _np(b["r"]))


@pytest.mark.parametrize("n", [64, 256, 4096])
def test_hadamard_exact_with_ties(n):
    """Sylvester columns (orthonormal, 1/sqrt(N) a power of two) and dyadic
    nonzeros: every sum is exact in FP32, so indices (equal |c| -> smaller
    index first, eq. 16), x~ and r are bit-exact."""
    s = _sylvester(n).T.copy()
    x = np.zeros(n, dtype=np.float32)
    x[[40, 5, 17, 3]] = [0.25, 0.5, -0.5, 0.125]
    y = mpgen.encode_signs(s, x)
    with _decoder(mpgen.pack_signs(s), n) as dec:
        g = _gpu_solver(dec, y)(0.0, 20, 20)
    assert g["idx"].tolist() == [5, 17, 40, 3]
    assert np.array_equal(g["x"], x) and not np.any(g["r"])
    assert g["stop"] == "converged"


def test_duplicate_and_negated_columns_tie_low():
    """N=6 gives 32 sign patterns up to sign, so M=300 columns repeat and
    negate each other.  Equal or opposite columns have |c| equal bit for bit,
    and the smallest index of the class is taken (eq. 16).  Expected: the
    oracle on the dictionary of class representatives (each class's smallest
    index), mapped back, up to its first step whose gap between classes is
    small."""
    rng = np.random.default_rng(4)
    n, m = 6, 300
    s = mpgen.bernoulli_signs(rng, n, m)
    canon = [tuple(int(v) for v in (s[j] * s[j][0])) for j in range(m)]
    first_of = {}
    for j, key in enumerate(canon):
        first_of.setdefault(key, j)
    reps = np.array(sorted(first_of.values()))
    y = rng.standard_normal(n).astype(np.float32)
    ora = osigns.solve_signs(mpgen.pack_signs(s[reps]), n, y, 1e-6, 30)
    with _decoder(mpgen.pack_signs(s), n) as dec:
        g = _gpu_solver(dec, y)(1e-6, 30, 30)
    assert set(g["idx"].tolist()) <= set(reps.tolist()), "a non-smallest member was selected"
    small = np.flatnonzero(ora.gap <= 1e-4 * np.sqrt(ora.yy))
    upto = int(small[0]) if small.size else ora.iters
    assert upto >= 3, upto
    assert g["idx"][:upto].tolist() == reps[ora.idx[:upto]].tolist()
    np.testing.assert_allclose(g["coef"][:upto], ora.coef[:upto], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("n,ldw", [(1, 1), (31, 2), (64, 2), (100, 5), (2049, 65), (8192, 256),
                                   (16383, 513)])
def test_storage_round_trip(n, ldw):
    """mp_get_storage returns the packed bits the context decodes: the input
    with its tail bits and spare words dropped, bit for bit."""
    rng = np.random.default_rng(n + ldw)
    m = 37
    raw = rng.integers(0, 2 ** 32, size=(m, ldw), dtype=np.uint64).astype(np.uint32)
    with _decoder(raw, n) as dec:
        codes, scales = dec.storage_copy()
    got = _np(codes).view(np.uint32)
    w = (n + 31) // 32
    want = raw[:, :w].copy()
    if n % 32:
        want[:, w - 1] &= np.uint32((1 << (n % 32)) - 1)
    assert scales is None and got.shape == (m, w)
    assert np.array_equal(got, want)


def test_stop_rules_and_rejects():
    from paper_0809_1833_amd import mp
    p = mpgen.make_sign_problem("c0", 5)
    with _decoder(p.bits, p.n) as dec:
        solve = _gpu_solver(dec, p.y)
        g = solve(1e-6, 0, 0)
        assert g["iters"] == 0 and g["stop"] == "max_iters"
        g = solve(2.0, 10, 0)
        assert g["iters"] == 0 and g["stop"] == "converged"
        g = solve(1e-6, 3, 3)
        ora = osigns.solve_signs(p.bits, p.n, p.y, 1e-6, 3)
        assert g["iters"] == 3 and g["stop"] == "max_iters"
        assert g["idx"].tolist() == ora.idx.tolist()
        g = _gpu_solver(dec, np.zeros(p.n, np.float32))(1e-6, 10, 0)
        assert g["iters"] == 0 and g["stop"] == "zero_input" and not np.any(g["x"])
        bad = p.y.copy()
        bad[7] = np.nan
        with pytest.raises(mp.MPError) as e:
            _gpu_solver(dec, bad)(1e-6, 10, 0)
        assert e.value.status == mp.MP_ENONFINITE
        yb = torch.from_numpy(np.tile(p.y[:, None], (1, 2)).T.copy()).cuda().t()
        with pytest.raises(mp.MPError) as e:
            dec.solve_batched(yb, 1e-6, 10)
        assert e.value.status == mp.MP_EINVAL
        with pytest.raises(mp.MPError) as e:
            mp.mp_solve_omp(dec.handle, torch.from_numpy(p.y).cuda().data_ptr(),
                            torch.empty(p.m, device="cuda").data_ptr(), None,
                            mp.Opts(1e-6, 10, 0, 0))
        assert e.value.status == mp.MP_EINVAL


def test_determinism():
    p = mpgen.make_sign_problem("c0", 6)
    with _decoder(p.bits, p.n) as dec:
        a = _gpu_solver(dec, p.y)(p.eps, p.max_iters, 50)
        b = _gpu_solver(dec, p.y)(p.eps, p.max_iters, 50)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["r"], b["r"])
