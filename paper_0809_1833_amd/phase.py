"""The reconstruction-error experiment of Fig. 1 (Section 3) on the batched
decoder.

E(sigma, rho) = ||x~ - x||^2 / ||x||^2 x 100 % on a grid of sigma = K/M and
rho = N/M, M = 1000, the +-1/sqrt(N) Bernoulli dictionary of eq. 13, nonzeros
drawn from U[-1, 1], eps = 1e-7 and T = N, averaged over the trials of each
cell.  For each rho the trials are split over ``draws`` dictionaries; every
draw decodes all sigmas' signals together with ``mp_solve_batched`` (one
shared dictionary per batch, the setting the batched form is built for).

Every decode runs in libmp; this module draws the inputs (``mpgen``), moves
them to the device and averages the error of the returned x~, an evaluation
of the result rather than part of the decode.
"""
from __future__ import annotations

import time
from typing import Callable, Optional, Sequence

import numpy as np
import torch

import mpgen
from .mp import Decoder


def grid(step: float = 0.05) -> list:
    """step, 2 step, ..., 1 (the axes of the figure)."""
    count = int(round(1.0 / step))
    return [round(step * i, 10) for i in range(1, count + 1)]


def _column_major(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def phase_diagram(rhos: Optional[Sequence[float]] = None,
                  sigmas: Optional[Sequence[float]] = None, trials: Optional[int] = None,
                  draws: Optional[int] = None, seed: int = 0, m: Optional[int] = None,
                  log: Optional[Callable[[str], None]] = None,
                  tile_rule: Optional[Sequence[int]] = None) -> dict:
    """E(sigma, rho) in percent on the grid, with per-cell mean iterations.
    ``tile_rule``: the batched product's switch points (Decoder.
    set_batched_config), else the library's default.

    Returns dict(rhos, sigmas, E (len(rhos) x len(sigmas)), iters (same
    shape), decodes, decode_seconds (device decode time only, input drawing
    excluded), signals_per_s)."""
    w = mpgen.workload("phase")
    rhos = grid() if rhos is None else list(rhos)
    sigmas = grid() if sigmas is None else list(sigmas)
    trials = w["trials"] if trials is None else int(trials)
    draws = w["draws"] if draws is None else int(draws)
    if trials % draws:
        raise ValueError("trials must be a multiple of draws")
    per_sigma = trials // draws
    e_sum = np.zeros((len(rhos), len(sigmas)))
    it_sum = np.zeros((len(rhos), len(sigmas)))
    decode_s, decodes = 0.0, 0
    for i, rho in enumerate(rhos):
        for d in range(draws):
            pb = mpgen.make_phase_batch(seed, rho, sigmas, d, per_sigma, m=m)
            x_true = torch.from_numpy(np.ascontiguousarray(pb.x.T)).cuda()  # (B, M)
            y = _column_major(pb.y)
            with Decoder(_column_major(pb.psi)) as dec:
                if tile_rule is not None:
                    dec.set_batched_config(*tile_rule)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = dec.solve_batched(y, pb.eps, pb.max_iters, want_r=False)
                torch.cuda.synchronize()
                decode_s += time.perf_counter() - t0
            xt = out["x"].t().to(torch.float64)                            # (B, M)
            xd = x_true.to(torch.float64)
            err = ((xt - xd) ** 2).sum(dim=1) / (xd ** 2).sum(dim=1) * 100.0
            err = err.cpu().numpy()
            iters = np.asarray(out["iters"], dtype=np.float64)
            np.add.at(e_sum[i], pb.sigma_index, err)
            np.add.at(it_sum[i], pb.sigma_index, iters)
            decodes += len(err)
        if log:
            log(f"[phase] rho={rho:.3f} done ({decodes} decodes, {decode_s:.2f} s on the device)")
    return dict(rhos=rhos, sigmas=sigmas, E=e_sum / trials, iters=it_sum / trials,
                decodes=decodes, decode_seconds=decode_s,
                signals_per_s=decodes / decode_s if decode_s > 0 else None)


def render(result: dict, levels: str = " .:-=+*#%@") -> str:
    """The diagram as text: rows rho (top = 1), columns sigma, darker = larger
    E (white 0 % to black 100 %, as in the figure)."""
    rows = []
    for i in range(len(result["rhos"]) - 1, -1, -1):
        cells = []
        for e in result["E"][i]:
            k = min(len(levels) - 1, int(round(float(e) / 100.0 * (len(levels) - 1))))
            cells.append(levels[k])
        rows.append(f"{result['rhos'][i]:5.2f} |" + "".join(cells) + "|")
    rows.append("       sigma = K/M ->")
    return "\n".join(rows)


if __name__ == "__main__":
    res = phase_diagram(log=print)
    print(render(res))
    print(f"{res['decodes']} decodes in {res['decode_seconds']:.2f} s "
          f"({res['signals_per_s']:.0f} signals/s)")
