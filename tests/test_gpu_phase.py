"""GPU checks of the Fig. 1 experiment driver (paper_0809_1833_amd.phase):
the batched decodes it makes agree with the FP64 oracle signal by signal, and
the diagram has the shape the paper reports (exact recovery at small sigma
and large rho, large error at large sigma and small rho)."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from parity import fp32_dot_bound
from wholerun import whole_run

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
    """Every signal of a Fig. 1 batch: the oracle's free run up to the first
    difference, which must be one the oracle's top-two gap allows (gap <=
    1e-5 ||r|| + 2 ||r_gpu - r_ora|| + 2 e32 on the state there), then every
    step of the GPU run on its own state and the oracle's replay of its atoms
    (x~ and r at the end within 1e-5)."""
    from paper_0809_1833_amd.mp import Decoder
    pb = mpgen.make_phase_batch(0, rho, SIGMAS, draw=0, per_sigma=3, m=M)
    n = pb.psi.shape[0]
    print(f"[phase rho={rho} N={n}]", flush=True)
    with Decoder(_cm(pb.psi)) as dec:
        out = dec.solve_batched(_cm(pb.y), pb.eps, pb.max_iters, trace_cap=n, trace_r=True)
        torch.cuda.synchronize()
    xg = out["x"].cpu().numpy()
    rg = out["r"].cpu().numpy()
    idx = out["idx"].cpu().numpy()
    coef = out["coef"].cpu().numpy()
    rtr = out["r_trace"].cpu().numpy()
    corr = oracle.Correlator(pb.psi)
    diverged = 0
    for j in range(pb.x.shape[1]):
        yj = pb.y[:, j]
        ora = oracle.solve(pb.psi, yj, pb.eps, pb.max_iters)
        k = out["iters"][j]
        g = idx[j, :k]
        L = min(k, ora.iters)
        diff = np.flatnonzero(g[:L] != ora.idx[:L])
        prefix = int(diff[0]) if diff.size else L
        if prefix < L:
            diverged += 1
            # the states of both runs before the differing step
            rep = oracle.replay(pb.psi, yj, g[:prefix], check_ties=False)
            r_o = rep.r if prefix else yj.astype(np.float64)
            r_g = rtr[j, prefix - 1].astype(np.float64) if prefix else yj.astype(np.float64)
            rn = float(np.linalg.norm(r_o))
            allowed = 1e-5 * rn + 2 * float(np.linalg.norm(r_g - r_o)) + 2 * fp32_dot_bound(n, rn)
            assert ora.gap[prefix] <= allowed, (j, prefix, ora.gap[prefix], allowed)
        gj = dict(x=xg[:, j], r=rg[:, j], iters=k, stop=out["stop"][j], idx=g,
                  coef=coef[j, :k], r_trace=rtr[j, :k])
        w = whole_run(pb.psi, yj, pb.eps, gj, corr=corr)
        assert w.misses == 0
        xt = pb.x[:, j].astype(np.float64)
        e_ora = float(np.sum((ora.x - xt) ** 2) / np.sum(xt ** 2) * 100)
        e_gpu = float(np.sum((xg[:, j] - xt) ** 2) / np.sum(xt ** 2) * 100)
        if e_ora < 1e-8:        # the oracle recovered x exactly: so must the GPU
            assert e_gpu < 1e-3, (j, e_gpu)
    print(f"[phase rho={rho}] {diverged} of {pb.x.shape[1]} signals leave the oracle's "
          f"free run at a near tie", flush=True)


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
