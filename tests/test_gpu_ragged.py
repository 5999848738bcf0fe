"""GPU parity of the ragged decoder (mp_create_ragged / mp_solve_ragged: many
independent problems of uneven size in one persistent, graph-replayed launch)
against the FP64 oracle, instance by instance."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from parity import run_parity
from wholerun import whole_run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(psi):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(psi, dtype=np.float32).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _ragged(probs, storage="f32"):
    from paper_0809_1833_amd.mp import RaggedDecoder
    return RaggedDecoder([_dev(p.psi) for p in probs], storage=storage)


def _ypacked(probs):
    return torch.from_numpy(np.concatenate([p.y for p in probs]).astype(np.float32)).cuda()


def _solve(dec, yp, eps, caps, cap):
    out = dec.solve(yp, eps, caps, trace_cap=cap)
    torch.cuda.synchronize()
    res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"])
    if cap:
        res.update(idx=_np(out["idx"]), coef=_np(out["coef"]), rr_trace=_np(out["rr_trace"]))
    return res


def _instance_solver(dec, yp, i, count):
    """gpu_solve for instance i: the whole set decoded, all other caps 0."""
    def solve(eps, max_iters, cap):
        caps = [0] * count
        caps[i] = max_iters
        g = _solve(dec, yp, eps, caps, cap)
        xs = slice(dec.x_off[i], dec.x_off[i + 1])
        ys = slice(dec.y_off[i], dec.y_off[i + 1])
        out = dict(x=g["x"][xs], r=g["r"][ys], iters=g["iters"][i], stop=g["stop"][i])
        k = g["iters"][i]
        if cap:
            out.update(idx=g["idx"][i, :k], coef=g["coef"][i, :k], rr_trace=g["rr_trace"][i, :k])
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


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_small_ragged_parity(storage):
    probs = mpgen.make_ragged(0, count=20, n_choices=(32, 64, 128, 256))
    eps = 1e-6
    with _ragged(probs, storage) as dec:
        yp = _ypacked(probs)
        for i, p in enumerate(probs):
            print(f"[{storage} instance {i} N={p.n}]", flush=True)
            rep = run_parity(p.psi, p.y, eps, p.max_iters, _instance_solver(dec, yp, i, len(probs)))
            assert rep.prefix >= min(rep.iters_ora, 20), (i, rep)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_ragged_workload_whole_run(storage):
    """The ragged workload: 512 instances, N in {128, 256, 512, 1024}, M = 4N,
    K = N/16, eps = 1e-5, T = 20K, in the benchmarked launch.  Every step of
    every instance against the FP64 oracle (the atom is the FP64 argmax of
    the instance's state wherever the top-two gap exceeds 1e-5 ||r||, the
    coefficient within the FP32 bound, each atom a near tie of the oracle's
    replayed state, x~ and r at the end within 1e-5 of the replay); every
    instance meets the stop rule and y = Psi x~ + r; six instances against
    the oracle's free run."""
    probs = mpgen.make_ragged(0)
    caps = [p.max_iters for p in probs]
    with _ragged(probs, storage) as dec:
        yp = _ypacked(probs)
        out = dec.solve(yp, 1e-5, caps, trace_cap=max(caps), trace_r=True)
        torch.cuda.synchronize()
        tot = dict(steps=0, exact=0, near_ties=0, misses=0, x_err=0.0, r_err=0.0)
        for i, p in enumerate(probs):
            k = out["iters"][i]
            gi = dict(x=_np(out["x"][dec.x_off[i]:dec.x_off[i + 1]]),
                      r=_np(out["r"][dec.y_off[i]:dec.y_off[i + 1]]), iters=k,
                      stop=out["stop"][i], idx=_np(out["idx"][i, :k]),
                      coef=_np(out["coef"][i, :k]), r_trace=_np(out["r_trace"][i, :k, :p.n]))
            w = whole_run(p.psi, p.y, 1e-5, gi)
            tot["steps"] += w.steps
            tot["exact"] += w.exact_steps
            tot["near_ties"] += w.near_ties
            tot["misses"] += w.misses
            tot["x_err"] = max(tot["x_err"], w.x_err)
            tot["r_err"] = max(tot["r_err"], w.r_err)
            if i % 64 == 0:
                print(f"[{storage} c4 whole run: instance {i} N={p.n}, {k} steps] {w}", flush=True)
        print(f"[{storage} c4 whole run] {tot}", flush=True)
        assert tot["misses"] == 0 and tot["steps"] == sum(out["iters"])
        del out
        g = _solve(dec, yp, 1e-5, caps, 0)
        for i, p in enumerate(probs):
            xs = g["x"][dec.x_off[i]:dec.x_off[i + 1]].astype(np.float64)
            rs = g["r"][dec.y_off[i]:dec.y_off[i + 1]].astype(np.float64)
            yn = np.linalg.norm(p.y.astype(np.float64))
            assert g["stop"][i] in ("converged", "max_iters"), i
            if g["stop"][i] == "converged":
                assert rs @ rs <= (1e-5 * yn) ** 2 * 1.000001, i
            defect = p.y - np.asarray(p.psi, np.float64) @ xs - rs
            assert np.linalg.norm(defect) <= 1e-5 * yn, i
        picks = [i for i, p in enumerate(probs) if p.n == 1024][:2] + \
                [i for i, p in enumerate(probs) if p.n == 512][:2] + \
                [i for i, p in enumerate(probs) if p.n == 128][:2]
        for i in picks:
            p = probs[i]
            print(f"[{storage} c4 instance {i} N={p.n}]", flush=True)
            rep = run_parity(p.psi, p.y, 1e-5, p.max_iters,
                             _instance_solver(dec, yp, i, len(probs)))
            assert rep.prefix >= min(rep.iters_ora, 50), (i, rep)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_launch_shape_does_not_change_selections(storage):
    """Every launch shape, and every split of the instances into parts (40
    instances on a grid of 256 or more workgroups: each exceeds the average
    work per workgroup, so each is cut into `split` parts that exchange
    their candidates every step), gives the same atoms, x~ and r bit for
    bit.  With BF16 storage the 1024-thread shapes score the short columns
    (N <= 256) with the wave-wide pass and the others side by side in lane
    groups, so the two passes are compared bit for bit too."""
    probs = mpgen.make_ragged(1, count=40, n_choices=(64, 128, 256, 512))
    caps = [p.max_iters for p in probs]
    with _ragged(probs, storage) as dec:
        yp = _ypacked(probs)
        dec.set_config(1024, 1, 1, 1)
        ref = _solve(dec, yp, 1e-5, caps, 64)
        shapes = [(256, 1, 1, 1), (512, 2, 2, 2), (1024, 4, 1, 4), (256, 4, 2, 8),
                  (1024, 1, 2, 3), (1024, 2, 1, 2), (512, 1, 1, 8)]
        for shape in shapes:
            print(f"[ragged {storage} shape {shape}]", flush=True)
            dec.set_config(*shape)
            assert dec.get_config() == dict(threads=shape[0], cols_per_wave=shape[1],
                                            wgs_per_cu=shape[2], split=shape[3])
            g = _solve(dec, yp, 1e-5, caps, 64)
            assert np.array_equal(g["idx"], ref["idx"]), shape
            assert np.array_equal(g["x"], ref["x"]), shape
            assert np.array_equal(g["r"], ref["r"]), shape
            assert g["iters"] == ref["iters"] and g["stop"] == ref["stop"], shape


def test_split_wait_limit_fails_cleanly(monkeypatch):
    """The waits between the parts of an instance allowed no poll
    (MP_RAGGED_SPIN_LIMIT=0, read at each call): the solve returns
    MP_EDEVICE, and the context then solves as before."""
    from paper_0809_1833_amd import mp
    probs = mpgen.make_ragged(5, count=16, n_choices=(128, 256))
    caps = [p.max_iters for p in probs]
    with _ragged(probs) as dec:
        yp = _ypacked(probs)
        dec.set_config(1024, 1, 1, 4)
        a = _solve(dec, yp, 1e-5, caps, 8)
        monkeypatch.setenv("MP_RAGGED_SPIN_LIMIT", "0")
        with pytest.raises(mp.MPError) as e:
            _solve(dec, yp, 1e-5, caps, 8)
        assert e.value.status == mp.MP_EDEVICE
        monkeypatch.delenv("MP_RAGGED_SPIN_LIMIT")
        b = _solve(dec, yp, 1e-5, caps, 8)
    assert np.array_equal(a["x"], b["x"]) and a["iters"] == b["iters"]


def test_graph_replay_and_recapture():
    probs = mpgen.make_ragged(2, count=12, n_choices=(64, 128))
    caps = [p.max_iters for p in probs]
    with _ragged(probs) as dec:
        yp = _ypacked(probs)
        a = _solve(dec, yp, 1e-5, caps, 32)
        b = _solve(dec, yp, 1e-5, caps, 32)      # replays the captured graph
        assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["idx"], b["idx"])
        c = _solve(dec, yp, 1e-3, caps, 32)      # new eps: captured again
        assert all(ci <= ai for ci, ai in zip(c["iters"], a["iters"]))
        d = _solve(dec, yp, 1e-5, caps, 32)
        assert np.array_equal(a["x"], d["x"])


def test_ragged_edge_cases():
    from paper_0809_1833_amd import mp
    probs = mpgen.make_ragged(3, count=5, n_choices=(16, 32))
    probs[2].y[:] = 0.0
    caps = [p.max_iters for p in probs]
    caps[3] = 0
    with _ragged(probs) as dec:
        g = _solve(dec, _ypacked(probs), 1e-6, caps, 16)
        assert g["stop"][2] == "zero_input" and g["iters"][2] == 0
        assert g["stop"][3] == "max_iters" and g["iters"][3] == 0
        with pytest.raises(mp.MPError) as e:
            dec.set_config(300, 1, 1)
        assert e.value.status == mp.MP_EINVAL
    # a 1-column instance and an n = 1 instance
    rng = np.random.default_rng(0)
    tiny = []
    for n, m in [(1, 1), (3, 1), (70, 5)]:
        psi = mpgen.gaussian_unit_dictionary(rng, n, m)
        x, sup = mpgen.sparse_signal(rng, rng, m, 1)
        tiny.append(mpgen.Problem(psi, x, mpgen.encode(psi, x, sup), sup, 1e-6, 20))
    with _ragged(tiny) as dec:
        g = _solve(dec, _ypacked(tiny), 1e-6, [20] * 3, 20)
        for i, p in enumerate(tiny):
            ora = oracle.solve(p.psi, p.y, 1e-6, 20)
            assert g["idx"][i, :g["iters"][i]].tolist()[:5] == ora.idx.tolist()[:5]


def test_ragged_rejects():
    from paper_0809_1833_amd import mp
    probs = mpgen.make_ragged(3, count=2, n_choices=(16,))
    with pytest.raises(mp.MPError) as e:
        _ragged(probs, "fp8")
    assert e.value.status == mp.MP_EUNSUPPORTED
    with _ragged(probs) as dec:
        opts = mp.Opts(1e-5, 10, 0, 0)
        x = torch.empty(64, device="cuda")
        y = torch.zeros(16, device="cuda")
        with pytest.raises(mp.MPError) as e:
            mp.mp_solve(dec.handle, y.data_ptr(), x.data_ptr(), None, opts)
        assert e.value.status == mp.MP_EINVAL


def test_autotuner_picks_a_valid_shape(tmp_path, monkeypatch):
    from paper_0809_1833_amd import tune
    monkeypatch.setenv("MP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs = mpgen.make_ragged(4, count=24, n_choices=(64, 128, 256))
    caps = [p.max_iters for p in probs]
    with _ragged(probs) as dec:
        yp = _ypacked(probs)
        res = tune.tune_ragged(dec, yp, 1e-5, caps, reps=1,
                               shapes=[(256, 1, 1), (1024, 2, 1), (512, 4, 2)])
        # three shapes at split 2, then the other splits on the best
        # (here all three)
        assert not res["cached"]
        assert len(res["timings"]) == 3 + min(3, tune.SPLIT_SHAPES) * (len(tune.SPLITS) - 1)
        assert dec.get_config() == res["config"]
        again = tune.tune_ragged(dec, yp, 1e-5, caps)
        assert again["cached"] and again["config"] == res["config"]
