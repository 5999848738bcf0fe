"""The one-launch FP32 decode of small dictionaries against the stepping form.

Where every workgroup's share of the columns fits in LDS (at most 32
workgroups, e.g. N=256, M=1024), mp_solve runs the whole decode in one
launch; with MP_SOLVE_STEP_LAUNCHES it takes one launch per iteration.  The
two run the same selection, update and correlation code, so every output
(x~, r, iterations, stop reason, the traced atoms, coefficients, norms and
residuals) must agree bit for bit.  Parity of the decode itself against the
FP64 oracle is covered by the FP32 tests, which at these sizes now run the
one-launch form.
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from parity import run_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _problem(case, seed=0):
    if case in ("c0", "c1a"):
        return mpgen.make_problem(case, seed)
    n, m = (int(v) for v in case.split("x"))
    rng = mpgen.rng_streams(77, seed + n * 7 + m, 3)
    psi = np.asfortranarray(mpgen.gaussian_unit_dictionary(rng[0], n, m))
    k = max(1, min(m, n) // 8)
    x, sup = mpgen.sparse_signal(rng[1], rng[2], m, k)
    return mpgen.Problem(psi, x, mpgen.encode(psi, x, sup), sup, 1e-6, 20 * k + 5)


def _decode(dec, y, p, cap, **kw):
    out = dec.solve(y, p.eps, p.max_iters, trace_cap=cap, trace_r=cap > 0, **kw)
    torch.cuda.synchronize()
    g = {k: out[k] for k in ("iters", "stop", "rr", "yy", "persistent")}
    for k in ("x", "r", "idx", "coef", "rr_trace", "r_trace"):
        if k in out:
            g[k] = _np(out[k]).copy()
    return g


@pytest.mark.parametrize("case", ["c0", "100x300", "1x5", "33x17", "2047x40", "256x4096",
                                  "64x2000", "1024x1000"])
def test_one_launch_matches_step_launches(case):
    from paper_0809_1833_amd.mp import Decoder
    p = _problem(case)
    print(f"[small one-launch {case}]", flush=True)
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(np.asarray(p.y, np.float32)).cuda()
    with Decoder(psi) as dec:
        a = _decode(dec, y, p, p.max_iters)
        b = _decode(dec, y, p, p.max_iters, step_launches=True)
        c = _decode(dec, y, p, 0)  # untraced
    assert a["persistent"] and not b["persistent"], (a["persistent"], b["persistent"])
    assert a["iters"] == b["iters"] == c["iters"] and a["stop"] == b["stop"] == c["stop"]
    assert a["rr"] == b["rr"] and a["yy"] == b["yy"]
    for key in ("x", "r", "idx", "coef", "rr_trace", "r_trace"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["x"], c["x"]) and np.array_equal(a["r"], c["r"])


def test_large_dictionary_steps():
    """A dictionary whose shares do not fit 32 workgroups' LDS steps."""
    from paper_0809_1833_amd.mp import Decoder
    p = mpgen.make_problem("c1a", 0)
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(p.y).cuda()
    with Decoder(psi) as dec:
        out = dec.solve(y, p.eps, 3)
    assert not out["persistent"]


def test_parity_c0_seeds():
    """N=256, M=1024 through the one-launch form against the FP64 oracle,
    three seeds: the index sequence, x~ and r at the prefix."""
    from paper_0809_1833_amd.mp import Decoder
    for seed in range(3):
        p = mpgen.make_problem("c0", seed)
        psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
        yd = torch.from_numpy(p.y).cuda()
        print(f"[small parity c0 seed {seed}]", flush=True)
        with Decoder(psi) as dec:
            def solve(eps, max_iters, cap):
                out = dec.solve(yd, eps, max_iters, trace_cap=cap)
                torch.cuda.synchronize()
                assert out["persistent"]
                res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"],
                           stop=out["stop"], rr=out["rr"], yy=out["yy"])
                if cap:
                    res.update(idx=_np(out["idx"]), coef=_np(out["coef"]),
                               rr_trace=_np(out["rr_trace"]))
                else:
                    res.update(idx=np.zeros(0, np.int32), coef=np.zeros(0, np.float32),
                               rr_trace=np.zeros(0))
                return res
            rep = run_parity(p.psi, p.y, p.eps, p.max_iters, solve)
        assert rep.full_match and rep.x_err <= 1e-5 and rep.r_err <= 1e-5, rep


def test_stop_rules():
    """Zero y (no step), a cap of 0 and of 3 steps, eps = 0 with a cap, and a
    NaN in y (MP_ENONFINITE): as the stepping form gives them."""
    from paper_0809_1833_amd import mp
    from paper_0809_1833_amd.mp import Decoder
    p = mpgen.make_problem("c0", 1)
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    with Decoder(psi) as dec:
        for yv, eps, cap in ((np.zeros_like(p.y), p.eps, 50), (p.y, p.eps, 0), (p.y, p.eps, 3),
                             (p.y, 0.0, 40)):
            q = mpgen.Problem(p.psi, p.x, yv, p.support, eps, cap)
            y = torch.from_numpy(np.ascontiguousarray(yv)).cuda()
            a = _decode(dec, y, q, max(cap, 1))
            b = _decode(dec, y, q, max(cap, 1), step_launches=True)
            assert a["iters"] == b["iters"] and a["stop"] == b["stop"], (cap, a["stop"], b["stop"])
            for key in ("x", "r", "idx", "coef"):
                assert np.array_equal(a[key], b[key]), key
        yn = p.y.copy()
        yn[7] = np.nan
        with pytest.raises(mp.MPError) as e:
            dec.solve(torch.from_numpy(yn).cuda(), p.eps, 50)
        assert e.value.status == mp.MP_ENONFINITE


def test_wait_limit_fails_cleanly(monkeypatch):
    """The one-launch decode's waits allowed no poll (MP_SMALL_SPIN_LIMIT=0,
    read at each decode): the first wait gives up in every workgroup, the
    decode returns MP_EDEVICE, and the context then decodes as before."""
    from paper_0809_1833_amd import mp
    from paper_0809_1833_amd.mp import Decoder
    p = mpgen.make_problem("c0", 0)
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(p.y).cuda()
    with Decoder(psi) as dec:
        monkeypatch.setenv("MP_SMALL_SPIN_LIMIT", "0")
        with pytest.raises(mp.MPError) as e:
            dec.solve(y, p.eps, p.max_iters)
        assert e.value.status == mp.MP_EDEVICE
        monkeypatch.delenv("MP_SMALL_SPIN_LIMIT")
        a = _decode(dec, y, p, 0)
        b = _decode(dec, y, p, 0, step_launches=True)
    assert a["persistent"] and a["iters"] == b["iters"] and np.array_equal(a["x"], b["x"])
