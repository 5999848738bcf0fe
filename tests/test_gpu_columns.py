"""Every column of a large dictionary is streamed exactly once: M of 16385
and 20001 give workgroup shares of several columns per wave and a ragged
last workgroup.

With y = psi_j for a random unit-norm dictionary, the first MP step (eq. 9)
must take j: |<psi_j, psi_j>| = 1 while every other |c| is far below 1 at
N = 64 (about 0.6 at most over 20k columns).  Sweeping j over the first and
last columns and a random sample covers the workgroups' shares, their
boundaries and the ragged tail; a skipped or doubled column would show as a
different index or coefficient.  Full parity against the FP64 oracle at the
same shapes follows."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
from parity import run_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(64, 20001), (33, 16385)]
STORAGES = ["f32", "bf16", "fp8"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()


def _dev(psi):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(psi, dtype=np.float32).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("n,m", SHAPES)
def test_single_atom_signal_selects_its_column(storage, n, m):
    from paper_0809_1833_amd.mp import Decoder
    rng = np.random.default_rng(m + n)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    js = sorted(set(range(16)) | set(range(m - 40, m)) |
                set(rng.choice(m, size=120, replace=False).tolist()))
    print(f"[columns {storage} {n}x{m}]", flush=True)
    with Decoder(_dev(psi), storage=storage) as dec:
        for j in js:
            y = torch.from_numpy(psi[:, j].copy()).cuda()
            out = dec.solve(y, 1e-12, 1, trace_cap=1)
            torch.cuda.synchronize()
            idx = int(_np(out["idx"])[0])
            assert idx == j, (j, idx)
            # the coefficient is the FP32 <psi_j, psi_j> (re-scored in FP32 for
            # the reduced-precision forms)
            np.testing.assert_allclose(_np(out["coef"])[0], 1.0, rtol=2e-6)


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("n,m", SHAPES)
def test_parity_large_m(storage, n, m):
    from paper_0809_1833_amd.mp import Decoder
    rng = np.random.default_rng(7 * m + n)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    x, sup = mpgen.sparse_signal(rng, rng, m, 4)
    y = mpgen.encode(psi, x, sup)
    yd = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()
    print(f"[parity {storage} {n}x{m}]", flush=True)

    with Decoder(_dev(psi), storage=storage) as dec:
        def solve(eps, max_iters, cap):
            out = dec.solve(yd, eps, max_iters, trace_cap=cap)
            torch.cuda.synchronize()
            res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                       rr=out["rr"], yy=out["yy"])
            if cap:
                res.update(idx=_np(out["idx"]), coef=_np(out["coef"]),
                           rr_trace=_np(out["rr_trace"]))
            else:
                res.update(idx=np.zeros(0, np.int32), coef=np.zeros(0, np.float32),
                           rr_trace=np.zeros(0))
            return res
        rep = run_parity(psi, y, 1e-6, 60, solve)
    print(rep, flush=True)
    assert rep.prefix >= min(rep.iters_ora, 10), rep


@pytest.mark.parametrize("n,m", [(256, 24576), (64, 16384)])
def test_parity_balanced_shares(n, m):
    """FP32 decodes whose passes split the columns by measured workgroup
    speed (256 workgroups of 96 and 64 columns on average): every pass after
    the first uses shares computed from the previous pass's timings, so a
    gap or overlap between workgroups' ranges would surface as a different
    selection over the 150 steps."""
    from paper_0809_1833_amd.mp import Decoder
    rng = np.random.default_rng(3 * m + n)
    psi = mpgen.gaussian_unit_dictionary(rng, n, m)
    x, sup = mpgen.sparse_signal(rng, rng, m, max(4, n // 16))
    y = mpgen.encode(psi, x, sup)
    yd = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()
    print(f"[balanced {n}x{m}]", flush=True)
    with Decoder(_dev(psi), storage="f32") as dec:
        def solve(eps, max_iters, cap):
            out = dec.solve(yd, eps, max_iters, trace_cap=cap)
            torch.cuda.synchronize()
            res = dict(x=_np(out["x"]), r=_np(out["r"]), iters=out["iters"], stop=out["stop"],
                       rr=out["rr"], yy=out["yy"])
            if cap:
                res.update(idx=_np(out["idx"]), coef=_np(out["coef"]),
                           rr_trace=_np(out["rr_trace"]))
            else:
                res.update(idx=np.zeros(0, np.int32), coef=np.zeros(0, np.float32),
                           rr_trace=np.zeros(0))
            return res
        rep = run_parity(psi, y, 1e-6, 150, solve)
        # decodes on the same context split their passes by their own
        # timings, which differ run to run; the results must not
        first = solve(1e-6, 150, 150)
        again = solve(1e-6, 150, 150)
    print(rep, flush=True)
    assert rep.prefix >= min(rep.iters_ora, 40), rep
    assert np.array_equal(first["idx"], again["idx"]) and np.array_equal(first["x"], again["x"])
    assert np.array_equal(first["r"], again["r"])
