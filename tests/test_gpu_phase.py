"""GPU checks of the Fig. 1 experiment driver (paper_0809_1833_amd.phase):
the batched decodes it makes agree with the FP64 oracle signal by signal, and
the diagram has the shape the paper reports (exact recovery at small sigma
and large rho, large error at large sigma and small rho)."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M = 200
RHOS = [0.1, 0.3, 0.6]
SIGMAS = [0.02, 0.1, 0.3]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0809_1833_amd import mp
    mp.library()


def _cm(a):
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


@pytest.mark.parametrize("rho", RHOS)
def test_batched_decodes_match_oracle(rho):
    from paper_0809_1833_amd.mp import Decoder
    pb = mpgen.make_phase_batch(0, rho, SIGMAS, draw=0, per_sigma=3, m=M)
    n = pb.psi.shape[0]
    print(f"[phase rho={rho} N={n}]", flush=True)
    with Decoder(_cm(pb.psi)) as dec:
        out = dec.solve_batched(_cm(pb.y), pb.eps, pb.max_iters, trace_cap=n, want_r=False)
        torch.cuda.synchronize()
    xg = out["x"].cpu().numpy()
    idx = out["idx"].cpu().numpy()
    full = 0
    for j in range(pb.x.shape[1]):
        ora = oracle.solve(pb.psi, pb.y[:, j], pb.eps, pb.max_iters)
        k = out["iters"][j]
        g = idx[j, :k]
        L = min(k, ora.iters)
        diff = np.flatnonzero(g[:L] != ora.idx[:L])
        prefix = int(diff[0]) if diff.size else L
        assert prefix >= min(ora.iters, 5), (j, prefix, ora.iters)
        if prefix == L and k == ora.iters:
            full += 1
        xt = pb.x[:, j].astype(np.float64)
        e_ora = float(np.sum((ora.x - xt) ** 2) / np.sum(xt ** 2) * 100)
        e_gpu = float(np.sum((xg[:, j] - xt) ** 2) / np.sum(xt ** 2) * 100)
        if e_ora < 1e-8:        # the oracle recovered x exactly: so must the GPU
            assert e_gpu < 1e-3, (j, e_gpu)
    assert full >= 0.7 * pb.x.shape[1], full


def test_phase_diagram_shape_and_consistency():
    from paper_0809_1833_amd import phase
    res = phase.phase_diagram(RHOS, SIGMAS, trials=4, draws=2, seed=0, m=M)
    E = np.asarray(res["E"])
    assert E.shape == (3, 3) and res["decodes"] == 36
    assert np.all(E >= 0) and np.all(np.isfinite(E))
    # small K, many projections: exact recovery; K > N: no recovery
    assert E[2, 0] < 1e-3
    assert E[0, 2] > 10.0
    # the cell means are the per-signal errors of the same decodes
    from paper_0809_1833_amd.mp import Decoder
    per = []
    for d in range(2):
        pb = mpgen.make_phase_batch(0, RHOS[1], SIGMAS, d, 2, m=M)
        with Decoder(_cm(pb.psi)) as dec:
            out = dec.solve_batched(_cm(pb.y), pb.eps, pb.max_iters, want_r=False)
        xg = out["x"].cpu().numpy().astype(np.float64)
        xt = pb.x.astype(np.float64)
        e = np.sum((xg - xt) ** 2, axis=0) / np.sum(xt ** 2, axis=0) * 100
        per.append((pb.sigma_index, e))
    cell = np.zeros(3)
    for sidx, e in per:
        np.add.at(cell, sidx, e)
    np.testing.assert_allclose(E[1], cell / 4, rtol=1e-9, atol=1e-12)
