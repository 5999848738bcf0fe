"""GPU parity of the batched decoder (mp_solve_batched: shared dictionary, BF16
matrix-core correlations, FP32 re-scoring, per-signal stopping with on-device
compaction of the active list) against the FP64 oracle, signal by signal."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from parity import run_parity
from wholerun import whole_run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    """(R, C) column-major numpy -> (R, C) column-major CUDA tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _decoder(psi, storage="bf16"):
    from paper_0809_1833_amd.mp import Decoder
    return Decoder(_dev(psi), storage=storage)


def _batched(dec, Y, eps, caps, cap):
    out = dec.solve_batched(_dev(Y), eps, caps, trace_cap=cap)
    torch.cuda.synchronize()
    res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"])
    if cap:
        res.update(idx=_np(out["idx"]), coef=_np(out["coef"]), rr_trace=_np(out["rr_trace"]))
    return res


def _single_from_batched(dec, y):
    """A gpu_solve callable for one signal, decoded through mp_solve_batched."""
    def solve(eps, max_iters, cap):
        g = _batched(dec, y[:, None], eps, [max_iters], cap)
        out = dict(x=g["x"][:, 0], r=g["r"][:, 0], iters=g["iters"][0], stop=g["stop"][0])
        if cap:
            k = g["iters"][0]
            out.update(idx=g["idx"][0, :k], coef=g["coef"][0, :k], rr_trace=g["rr_trace"][0, :k])
        else:
            out.update(idx=np.zeros(0, np.int32), coef=np.zeros(0, np.float32),
                       rr_trace=np.zeros(0))
        return out
    return solve


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()


@pytest.mark.parametrize("storage", ["bf16", "f32"])
def test_small_batch_parity(storage):
    """N=256, M=1024, 12 signals with K_b in 2..20; every signal checked."""
    bt = mpgen.make_batch(0, b=12, n=256, m=1024, kmin=2, kmax=20)
    eps = 1e-6
    with _decoder(bt.psi, storage) as dec:
        g = _batched(dec, bt.y, eps, list(bt.max_iters), int(bt.max_iters.max()))
        for b in range(bt.y.shape[1]):
            print(f"[signal {b}]", flush=True)
            rep = run_parity(bt.psi, bt.y[:, b], eps, int(bt.max_iters[b]),
                             _single_from_batched(dec, bt.y[:, b]))
            assert rep.prefix >= min(rep.iters_ora, 30), (b, rep)
            # the signal's trajectory does not depend on the rest of the batch
            k = g["iters"][b]
            solo = _single_from_batched(dec, bt.y[:, b])(eps, int(bt.max_iters[b]), k)
            assert np.array_equal(g["idx"][b, :k], solo["idx"])
            assert np.array_equal(g["x"][:, b], solo["x"])


def test_batched_workload_whole_run():
    """The batched workload: N=2048, M=8192, B=256, K_b ~ U{16..256}, eps=1e-5,
    T_b = 20 K_b, decoded as one batch (the benchmarked launch sequence).
    Every step of every one of the 256 signals is checked against the FP64
    oracle: the re-scored atom is the FP64 argmax of the signal's state
    wherever the top-two gap exceeds 1e-5 ||r|| (no rescore misses), the
    coefficient within the FP32 bound, and the oracle's replay of the
    signal's atoms ends within 1e-5 of its x~ and r.  (The replay's own
    near-tie check follows from these through the bound |c^o - c^g| <=
    ||r^o - r^g|| and is not computed again here.)  Four signals also against
    the oracle's free run, and all 256 for the stop rule and y = Psi x~ + r."""
    bt = mpgen.make_batch(0)
    with _decoder(bt.psi) as dec:
        cap = int(bt.max_iters.max())
        out = dec.solve_batched(_dev(bt.y), bt.eps, list(bt.max_iters), trace_cap=cap,
                                trace_r=True)
        torch.cuda.synchronize()
        corr = oracle.Correlator(bt.psi)
        worst = dict(misses=0, near_ties=0, steps=0, x_err=0.0, r_err=0.0, exact=0)
        for b in range(bt.y.shape[1]):
            k = out["iters"][b]
            gb = dict(x=_np(out["x"][:, b]), r=_np(out["r"][:, b]), iters=k, stop=out["stop"][b],
                      idx=_np(out["idx"][b, :k]), coef=_np(out["coef"][b, :k]),
                      r_trace=_np(out["r_trace"][b, :k]))
            w = whole_run(bt.psi, bt.y[:, b], bt.eps, gb, oracle_ties=False, corr=corr)
            worst["misses"] += w.misses
            worst["near_ties"] += w.near_ties
            worst["steps"] += w.steps
            worst["exact"] += w.exact_steps
            worst["x_err"] = max(worst["x_err"], w.x_err)
            worst["r_err"] = max(worst["r_err"], w.r_err)
            if b % 32 == 0:
                print(f"[c3 whole run: signal {b}, {k} steps] {w}", flush=True)
        print(f"[c3 whole run] {worst}", flush=True)
        assert worst["misses"] == 0 and worst["steps"] == sum(out["iters"])
        del out
        g = _batched(dec, bt.y, bt.eps, list(bt.max_iters), 0)
        psi64 = np.asarray(bt.psi, dtype=np.float64)
        ynorm = np.linalg.norm(bt.y.astype(np.float64), axis=0)
        defect = bt.y - psi64 @ g["x"] - g["r"]
        assert np.all(np.linalg.norm(defect, axis=0) <= 1e-5 * ynorm)
        for b in range(bt.y.shape[1]):
            assert g["stop"][b] in ("converged", "max_iters")
            if g["stop"][b] == "converged":
                assert np.sum(g["r"][:, b].astype(np.float64) ** 2) <= (bt.eps * ynorm[b]) ** 2 * 1.000001
        for b in (0, 1, 100, 255):
            print(f"[c3 signal {b} K={bt.k[b]}]", flush=True)
            rep = run_parity(bt.psi, bt.y[:, b], bt.eps, int(bt.max_iters[b]),
                             _single_from_batched(dec, bt.y[:, b]))
            print(rep, flush=True)
            assert rep.prefix >= min(rep.iters_ora, 100)


NEVER = 2**31 - 1


@pytest.mark.parametrize("rule", [(0, 0, 0), (0, NEVER, 0), (NEVER, 0, 0), (NEVER, NEVER, 0),
                                  (NEVER, NEVER, NEVER), (100, 40, 12)])
def test_batched_tile_rules(rule):
    """Every tile rule of the batched product -- 128 atoms on eight waves, 64
    staged, 32, 16, and a rule that switches tiles as signals stop --
    decodes 160 signals with every step judged by the FP64 oracle (no
    selection off the FP64 argmax where the gap exceeds 1e-5 ||r||, x~ and r
    within 1e-5 of the oracle's replay).  M = 11000 leaves a ragged last
    tile for each tile height and gives even the 128-atom tile a workgroup
    for every CU at 160 signals; N = 512 lets the staged forms run."""
    bt = mpgen.make_batch(5, b=160, n=512, m=11000, kmin=2, kmax=8)
    eps = 1e-5
    with _decoder(bt.psi) as dec:
        dec.set_batched_config(*rule)
        assert dec.get_batched_config() == dict(atoms128_above=rule[0], atoms64_above=rule[1],
                                                atoms32_above=rule[2])
        cap = int(bt.max_iters.max())
        out = dec.solve_batched(_dev(bt.y), eps, list(bt.max_iters), trace_cap=cap, trace_r=True)
        torch.cuda.synchronize()
    corr = oracle.Correlator(bt.psi)
    misses = steps = 0
    xe = re = 0.0
    for b in range(bt.y.shape[1]):
        k = out["iters"][b]
        gb = dict(x=_np(out["x"][:, b]), r=_np(out["r"][:, b]), iters=k, stop=out["stop"][b],
                  idx=_np(out["idx"][b, :k]), coef=_np(out["coef"][b, :k]),
                  r_trace=_np(out["r_trace"][b, :k]))
        w = whole_run(bt.psi, bt.y[:, b], eps, gb, oracle_ties=False, corr=corr)
        misses += w.misses
        steps += w.steps
        xe, re = max(xe, w.x_err), max(re, w.r_err)
    print(f"[tile rule {rule}] steps {steps} misses {misses} x {xe:.2e} r {re:.2e}", flush=True)
    assert misses == 0 and steps == sum(out["iters"])
    assert xe <= 1e-5 and re <= 1e-5


def test_batched_tuner(tmp_path, monkeypatch):
    """The tuner times the rules it is given, applies the fastest, caches it."""
    from paper_0809_1833_amd import tune
    monkeypatch.setenv("MP_TUNE_CACHE", str(tmp_path / "tune.json"))
    bt = mpgen.make_batch(2, b=40, n=256, m=1024, kmin=2, kmax=8)
    caps = list(bt.max_iters)
    with _decoder(bt.psi) as dec:
        Y = _dev(bt.y)
        res = tune.tune_batched(dec, Y, 1e-5, caps, reps=1,
                                rules=[(NEVER, NEVER, 0), (NEVER, 16, 0), (16, 16, 8)])
        assert not res["cached"] and len(res["timings"]) == 3
        assert dec.get_batched_config() == res["config"]
        again = tune.tune_batched(dec, Y, 1e-5, caps)
        assert again["cached"] and again["config"] == res["config"]


def test_batched_config_errors():
    from paper_0809_1833_amd import mp
    bt = mpgen.make_batch(1, b=2, n=64, m=256, kmin=2, kmax=4)
    with _decoder(bt.psi) as dec:
        default = dict(atoms128_above=NEVER, atoms64_above=96, atoms32_above=0)
        assert dec.get_batched_config() == default
        for bad in [(-1, 5, 0), (5, 5, -1)]:
            with pytest.raises(mp.MPError) as e:
                dec.set_batched_config(*bad)
            assert e.value.status == mp.MP_EINVAL
        assert dec.get_batched_config() == default


def test_mixed_stops_and_caps():
    """Zero signals, zero caps, tiny caps and normal signals in one batch."""
    bt = mpgen.make_batch(3, b=9, n=250, m=1000, kmin=3, kmax=8)
    Y = bt.y.copy(order="F")
    Y[:, 2] = 0.0
    caps = [50, 50, 50, 0, 3, 50, 1, 50, 50]
    with _decoder(bt.psi) as dec:
        g = _batched(dec, Y, 1e-6, caps, 50)
    assert g["stop"][2] == "zero_input" and g["iters"][2] == 0 and not g["x"][:, 2].any()
    assert g["iters"][3] == 0 and g["stop"][3] == "max_iters"
    assert g["iters"][4] == 3 and g["stop"][4] == "max_iters"
    assert g["iters"][6] == 1
    for b in (0, 1, 5, 7, 8):
        ora = oracle.solve(bt.psi, Y[:, b], 1e-6, caps[b])
        k = min(g["iters"][b], ora.iters, 20)
        assert g["idx"][b, :k].tolist() == ora.idx[:k].tolist()


@pytest.mark.parametrize("n,m,b", [(3, 5, 2), (64, 130, 70), (16384, 64, 3), (520, 300, 5),
                                   (256, 1000, 130), (512, 4096, 100), (256, 16000, 100)])
def test_batched_shapes(n, m, b):
    """Ragged and extreme shapes.  The last three keep more than 96 signals
    active with column lengths a multiple of 256; the first two of them have
    too few atom tiles for the 64-atom tile to give every CU a workgroup, so
    they run 32-atom tiles, the last one runs the 64-atom product with the
    residual operand staged in LDS (a ragged last atom tile)."""
    rng = np.random.default_rng(n + m + b)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    Y = np.zeros((n, b), np.float32, order="F")
    for j in range(b):
        k = max(1, min(m // 8, n // 4, 5))
        x, sup = mpgen.sparse_signal(rng, rng, m, k)
        Y[:, j] = mpgen.encode(psi, x, sup)
    with _decoder(psi) as dec:
        g = _batched(dec, Y, 1e-6, [200] * b, 200)
        for j in range(b):
            ora = oracle.solve(psi, Y[:, j], 1e-6, 200)
            k = min(g["iters"][j], ora.iters, 15)
            assert g["idx"][j, :k].tolist() == ora.idx[:k].tolist(), j


def test_hadamard_ties_batched():
    psi = mpgen.hadamard_dictionary(16)
    x = np.zeros(16, np.float32)
    x[[3, 7, 11, 12, 14, 15]] = [-0.5, 0.5, 0.5, 0.25, -0.25, 0.125]
    y = mpgen.encode(psi, x)
    Y = np.stack([y, -y], axis=1).astype(np.float32, order="F")
    with _decoder(psi) as dec:
        g = _batched(dec, Y, 0.0, [20, 20], 20)
    assert g["idx"][0, :6].tolist() == [3, 7, 11, 12, 14, 15]
    assert g["idx"][1, :6].tolist() == [3, 7, 11, 12, 14, 15]
    assert g["coef"][0, :6].tolist() == [-0.5, 0.5, 0.5, 0.25, -0.25, 0.125]
    assert np.array_equal(g["x"][:, 0], x) and np.array_equal(g["x"][:, 1], -x)


def test_batched_errors():
    from paper_0809_1833_amd import mp
    bt = mpgen.make_batch(1, b=3, n=64, m=256, kmin=2, kmax=4)
    Y = bt.y.copy(order="F")
    Y[5, 1] = np.nan
    with _decoder(bt.psi) as dec:
        with pytest.raises(mp.MPError) as e:
            dec.solve_batched(_dev(Y), 1e-6, 50)
        assert e.value.status == mp.MP_ENONFINITE
        with pytest.raises(mp.MPError) as e:
            dec.solve_batched(_dev(bt.y), 1e-6, [5, -1, 5])
        assert e.value.status == mp.MP_EINVAL
        out = dec.solve_batched(_dev(bt.y), 1e-6, 50)
        assert all(s == "converged" for s in out["stop"])
