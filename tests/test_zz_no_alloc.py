"""The no-allocation decode (mp_solve_noalloc) against mp_solve, through the
C ABI.

mp_solve_noalloc runs the same kernels as mp_solve with the decode's work
buffers in the library's static device scratch instead of the context's own,
so its results must equal mp_solve's bit for bit (x~, r, iterations, stop
reason, the traced atoms, coefficients and norms).  Calls come in a row on
problems of decreasing size, so each call finds the scratch as a larger
earlier decode left it; the device's free memory must not change across
them.
"""
from __future__ import annotations

import numpy as np
import pytest

import mpgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _decode(dec, y, p, noalloc, x, r):
    out = dec.solve(y, p.eps, p.max_iters, x=x, r=r, trace_cap=p.max_iters, noalloc=noalloc)
    torch.cuda.synchronize()
    return {"x": _np(out["x"]).copy(), "r": _np(out["r"]).copy(), "iters": out["iters"],
            "stop": out["stop"], "rr": out["rr"], "yy": out["yy"], "idx": _np(out["idx"]).copy(),
            "coef": _np(out["coef"]).copy(), "rr_trace": _np(out["rr_trace"]).copy()}


def _same(a, b):
    assert a["iters"] == b["iters"] and a["stop"] == b["stop"], (a["iters"], b["iters"])
    assert a["rr"] == b["rr"] and a["yy"] == b["yy"]
    for k in ("x", "r", "idx", "coef", "rr_trace"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("storages", [("f32", "f32"), ("bf16", "fp8")])
def test_noalloc_equals_mp_solve_on_two_calls_in_a_row(storages):
    """First call: N=2048, M=8192, K=128; second call: N=256, M=1024, K=10
    (smaller, on a second context); each equals mp_solve on its context."""
    from paper_0809_1833_amd.mp import Decoder
    free_before = None
    for name, storage in zip(("c1a", "c0"), storages):
        p = mpgen.make_problem(name, 1)
        print(f"[noalloc] {name} {storage}", flush=True)
        psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
        y = torch.from_numpy(p.y).cuda()
        x = torch.empty(p.m, dtype=torch.float32, device="cuda")
        r = torch.empty(p.n, dtype=torch.float32, device="cuda")
        with Decoder(psi, storage=storage) as dec:
            ref = _decode(dec, y, p, False, x, r)
            torch.cuda.synchronize()
            free_a = torch.cuda.mem_get_info()[0]
            got = _decode(dec, y, p, True, x, r)
            again = _decode(dec, y, p, True, x, r)
            free_b = torch.cuda.mem_get_info()[0]
        _same(got, ref)
        _same(again, ref)
        assert free_a == free_b, "device memory changed across mp_solve_noalloc calls"
        assert ref["iters"] > 0 and ref["stop"] in ("converged", "max_iters")
        if free_before is None:
            free_before = free_a


def test_noalloc_after_other_contexts_and_stop_rules():
    """A zero y (no step), then a decode capped at 3 steps, then a full one,
    on one context: each as mp_solve gives it."""
    from paper_0809_1833_amd.mp import Decoder
    p = mpgen.make_problem("c0", 2)
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    x = torch.empty(p.m, dtype=torch.float32, device="cuda")
    r = torch.empty(p.n, dtype=torch.float32, device="cuda")
    with Decoder(psi, storage="f32") as dec:
        for yv, cap in ((np.zeros_like(p.y), p.max_iters), (p.y, 3), (p.y, p.max_iters)):
            q = mpgen.Problem(p.psi, p.x, yv, p.support, p.eps, cap)
            y = torch.from_numpy(np.ascontiguousarray(yv)).cuda()
            print(f"[noalloc] c0 cap {cap} zero={not yv.any()}", flush=True)
            _same(_decode(dec, y, q, True, x, r), _decode(dec, y, q, False, x, r))
