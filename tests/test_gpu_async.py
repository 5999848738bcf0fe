"""Stream-ordered decodes (MP_SOLVE_ASYNC) against the ordinary call.

A stream-ordered decode enqueues the same kernels as mp_solve (every launch
the cap allows instead of chunks cut by the host's readings of the state),
so x~, r, the trace and the result collected with mp_solve_result must equal
the ordinary decode's bit for bit.  Parity of the decode itself against the
FP64 oracle is covered by the FP32, precision and small-form tests.
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen

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


def _problem(case, seed=0):
    if case == "c0":
        return mpgen.make_problem("c0", seed)
    n, m = (int(v) for v in case.split("x"))
    rng = mpgen.rng_streams(78, seed + n * 7 + m, 3)
    psi = np.asfortranarray(mpgen.gaussian_unit_dictionary(rng[0], n, m))
    k = max(1, min(m, n) // 16)
    x, sup = mpgen.sparse_signal(rng[1], rng[2], m, k)
    return mpgen.Problem(psi, x, mpgen.encode(psi, x, sup), sup, 1e-6, 20 * k + 5)


def _dev(p):
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(np.asarray(p.y, np.float32)).cuda()
    return psi, y


def _sync(dec, y, p, **kw):
    out = dec.solve(y, p.eps, p.max_iters, trace_cap=p.max_iters, **kw)
    torch.cuda.synchronize()
    k = out["iters"]
    return dict(x=_np(out["x"]), r=_np(out["r"]), iters=k, stop=out["stop"], rr=out["rr"],
                yy=out["yy"], persistent=out["persistent"], idx=_np(out["idx"])[:k],
                coef=_np(out["coef"])[:k], rr_trace=_np(out["rr_trace"])[:k])


def _issue(dec, y, p, stream, **kw):
    """Enqueue a stream-ordered decode on `stream`; returns its output tensors."""
    stream.wait_stream(torch.cuda.current_stream())
    return dec.solve(y, p.eps, p.max_iters, trace_cap=p.max_iters, stream=stream,
                     asynchronous=True, **kw)


def _collect(dec, out):
    res = dec.result()
    torch.cuda.synchronize()
    k = res["iters"]
    return dict(x=_np(out["x"]), r=_np(out["r"]), iters=k, stop=res["stop"], rr=res["rr"],
                yy=res["yy"], persistent=res["persistent"], idx=_np(out["idx"])[:k],
                coef=_np(out["coef"])[:k], rr_trace=_np(out["rr_trace"])[:k])


def _same(a, b):
    for key in ("iters", "stop", "rr", "yy", "persistent"):
        assert a[key] == b[key], key
    for key in ("x", "r", "idx", "coef", "rr_trace"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("case,storage,kw", [
    ("c0", "f32", {}),                          # one launch, shares in LDS
    ("c0", "f32", {"step_launches": True}),     # one launch per step
    ("512x3000", "f32", {}),                    # too large for LDS: stepping
    ("1024x4096", "bf16", {}),
    ("1024x4096", "fp8", {}),
    ("512x3000", "f32", {"noalloc": True}),
    ("c0", "f32", {"noalloc": True}),
])
def test_async_matches_sync(case, storage, kw):
    from paper_0809_1833_amd.mp import Decoder
    p = _problem(case)
    print(f"[async {case} {storage} {kw}]", flush=True)
    psi, y = _dev(p)
    side = torch.cuda.Stream()
    with Decoder(psi, storage=storage) as dec:
        a = _sync(dec, y, p, **kw)
        out = _issue(dec, y, p, side, **kw)
        b = _collect(dec, out)
    _same(a, b)


def test_async_decodes_overlap_on_two_streams():
    """Two contexts, each with its decode issued on its own stream before
    either is collected; each result equals the ordinary decode's."""
    from paper_0809_1833_amd.mp import Decoder
    ps = [_problem("c0", 1), _problem("512x3000", 2)]
    devs = [_dev(p) for p in ps]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    decs = [Decoder(psi) for psi, _ in devs]
    try:
        ref = [_sync(d, y, p) for d, (_, y), p in zip(decs, devs, ps)]
        outs = [_issue(d, y, p, s) for d, (_, y), p, s in zip(decs, devs, ps, streams)]
        got = [_collect(d, o) for d, o in zip(decs, outs)]
    finally:
        for d in decs:
            d.close()
    for a, b in zip(ref, got):
        _same(a, b)


def test_async_cap_zero_and_zero_input():
    from paper_0809_1833_amd.mp import Decoder
    p = _problem("512x3000")
    psi, y = _dev(p)
    side = torch.cuda.Stream()
    with Decoder(psi) as dec:
        side.wait_stream(torch.cuda.current_stream())
        out = dec.solve(y, p.eps, 0, stream=side, asynchronous=True)
        res = dec.result()
        assert res["iters"] == 0 and res["stop"] == "max_iters"
        assert not _np(out["x"]).any() and np.array_equal(_np(out["r"]), p.y)
        z = torch.zeros_like(y)
        out = dec.solve(z, p.eps, 50, stream=side, asynchronous=True)
        res = dec.result()
        assert res["iters"] == 0 and res["stop"] == "zero_input"


def test_async_errors():
    from paper_0809_1833_amd import mp
    from paper_0809_1833_amd.mp import Decoder
    p = _problem("c0")
    psi, y = _dev(p)
    x = torch.empty(p.m, dtype=torch.float32, device="cuda")
    r = torch.empty(p.n, dtype=torch.float32, device="cuda")
    with Decoder(psi) as dec:
        opts = mp.Opts(p.eps, p.max_iters, 0, mp.MP_SOLVE_ASYNC)
        # res must be NULL
        with pytest.raises(mp.MPError) as e:
            mp.mp_solve(dec.handle, y.data_ptr(), x.data_ptr(), r.data_ptr(), opts)
        assert e.value.status == mp.MP_EINVAL
        # nothing pending
        with pytest.raises(mp.MPError) as e:
            dec.result()
        assert e.value.status == mp.MP_EINVAL
        # one pending decode per context: every decode call is refused until
        # the result is collected
        dec.solve(y, p.eps, p.max_iters, x=x, r=r, asynchronous=True)
        with pytest.raises(mp.MPError) as e:
            dec.solve(y, p.eps, p.max_iters, x=x, r=r)
        assert e.value.status == mp.MP_EINVAL
        with pytest.raises(mp.MPError) as e:
            dec.solve(y, p.eps, p.max_iters, x=x, r=r, asynchronous=True)
        assert e.value.status == mp.MP_EINVAL
        with pytest.raises(mp.MPError) as e:
            dec.solve_batched(y[:, None], p.eps, 10)
        assert e.value.status == mp.MP_EINVAL
        assert dec.result()["stop"] == "converged"
        # an error only the device finds comes back from the result call
        bad = y.clone()
        bad[3] = float("nan")
        dec.solve(bad, p.eps, p.max_iters, x=x, r=r, asynchronous=True)
        with pytest.raises(mp.MPError) as e:
            dec.result()
        assert e.value.status == mp.MP_ENONFINITE
        # and the context decodes again
        assert dec.solve(y, p.eps, p.max_iters, x=x, r=r)["stop"] == "converged"
        # closing with a decode pending waits for it
        dec.solve(y, p.eps, p.max_iters, x=x, r=r, asynchronous=True)
    torch.cuda.synchronize()
