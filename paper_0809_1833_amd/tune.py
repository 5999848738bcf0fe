"""Autotuners for the ragged decode's launch shape and the batched product's tiles.

The ragged decode (``mp_solve_ragged``) runs one persistent launch whose
shape -- workgroup size, columns streamed per wave, workgroups per CU, and
the most parts one large instance is cut into -- changes speed but never
results.  ``tune_ragged`` times every valid shape on the actual instances
(at split 2), then the other split choices on the six fastest
shapes, and keeps the fastest; the choice is cached in a JSON file keyed by the GPU
architecture, the storage type and the multiset of instance sizes, so later
runs with the same shape of work reuse it.

The batched decode (``mp_solve_batched``) picks the product's tile every
round from the number of signals still active: 128, 64, 32 or 16 atoms per
workgroup.  ``tune_batched`` times whole batched decodes under each rule of
a small grid of the 128- and 64-atom switch points, then the 16-atom switch
points on the fastest, and keeps the fastest, cached by architecture,
dictionary shape, batch size and the multiset of per-signal caps.

Cache file: ``$MP_TUNE_CACHE`` if set, else ``~/.cache/mp_mi355x_tune.json``.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from collections import Counter
from typing import Iterable, Optional

import torch

FP32_SHAPES = [(t, c, w) for t in (256, 512, 1024) for c in (1, 2, 4) for w in (1, 2)]
BF16_SHAPES = FP32_SHAPES
SPLITS = (1, 2, 3, 4)
RANK_SPLIT = 2  # the split every shape is first timed at
SPLIT_SHAPES = 6  # shapes whose other splits are timed too


def cache_path() -> str:
    return os.environ.get("MP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mp_mi355x_tune.json"))


def workload_key(dec, arch: Optional[str] = None) -> str:
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sizes = sorted(Counter(zip(dec.ns, dec.ms)).items())
    digest = hashlib.sha256(json.dumps(sizes).encode()).hexdigest()[:16]
    return f"{arch}|{dec.storage}|{dec.count}|{digest}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs a re-tune next time


def tune_ragged(dec, y_packed: torch.Tensor, eps: float, max_iters, reps: int = 2,
                shapes: Optional[Iterable] = None, use_cache: bool = True, log=None) -> dict:
    """Time each launch shape on this workload, apply and return the fastest.

    Returns dict(config=..., ms=..., timings=[...], cached=bool)."""
    key = workload_key(dec)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache and "split" in cache[key]["config"]:
        cfg = cache[key]["config"]
        dec.set_config(cfg["threads"], cfg["cols_per_wave"], cfg["wgs_per_cu"], cfg["split"])
        return dict(cache[key], cached=True)
    if shapes is None:
        shapes = BF16_SHAPES if dec.storage == "bf16" else FP32_SHAPES
    timings = []
    x = torch.empty(dec.x_off[-1], dtype=torch.float32, device=y_packed.device)

    def time_shape(t, c, w, sp):
        dec.set_config(t, c, w, sp)
        dec.solve(y_packed, eps, max_iters, want_r=False, x_out=x)  # capture + warm-up
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            dec.solve(y_packed, eps, max_iters, want_r=False, x_out=x)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        timings.append(dict(threads=t, cols_per_wave=c, wgs_per_cu=w, split=sp,
                            ms=round(best * 1e3, 3)))
        if log:
            log(f"[tune] threads={t} cols/wave={c} wgs/cu={w} split={sp}: {best * 1e3:.2f} ms")

    for (t, c, w) in shapes:
        time_shape(t, c, w, RANK_SPLIT)
    # the other splits on the best few shapes: the best split depends on the
    # shape (shapes that tie at split 2 can part at another)
    ranked = sorted(timings, key=lambda d: d["ms"])[:SPLIT_SHAPES]
    for d in ranked:
        for sp in SPLITS:
            if sp != RANK_SPLIT:
                time_shape(d["threads"], d["cols_per_wave"], d["wgs_per_cu"], sp)
    win = min(timings, key=lambda d: d["ms"])
    cfg = dict(threads=win["threads"], cols_per_wave=win["cols_per_wave"],
               wgs_per_cu=win["wgs_per_cu"], split=win["split"])
    dec.set_config(**cfg)
    entry = dict(config=cfg, ms=win["ms"], timings=timings)
    if use_cache:
        cache[key] = entry
        _store_cache(cache)
    return dict(entry, cached=False)


NEVER = 2**31 - 1  # a switch point no active count exceeds: the tile is not used
ATOMS128_ABOVE = (64, 128, 192, NEVER)
ATOMS64_ABOVE = (32, 64, 96, 160, NEVER)
ATOMS32_ABOVE = (16, 32, 64)  # tried on the fastest pair; 0 (no 16-atom tile) first


def batched_key(dec, n_signals: int, max_iters, arch: Optional[str] = None) -> str:
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    caps = [int(v) for v in max_iters] if hasattr(max_iters, "__len__") else [int(max_iters)]
    digest = hashlib.sha256(json.dumps(sorted(Counter(caps).items())).encode()).hexdigest()[:16]
    return f"batched|{arch}|{dec.n}|{dec.m}|{n_signals}|{digest}"


def batched_rules():
    """The switch-point pairs tried first (no 16-atom tile): a 64-atom
    switch at or below the 128-atom one (above it the 64-atom tile would
    never run), or none."""
    return [(a128, a64, 0) for a128 in ATOMS128_ABOVE for a64 in ATOMS64_ABOVE
            if a64 <= a128 or a64 == NEVER]


def tune_batched(dec, Y: torch.Tensor, eps: float, max_iters, reps: int = 2,
                 rules: Optional[Iterable] = None, use_cache: bool = True, log=None) -> dict:
    """Time whole batched decodes of Y under each tile rule (triples of
    switch points; by default batched_rules(), then ATOMS32_ABOVE on the
    fastest), apply and return the fastest: dict(config=..., ms=...,
    timings=[...], cached=bool)."""
    key = batched_key(dec, Y.shape[1], max_iters)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache and "atoms32_above" in cache[key]["config"]:
        cfg = cache[key]["config"]
        dec.set_batched_config(cfg["atoms128_above"], cfg["atoms64_above"], cfg["atoms32_above"])
        return dict(cache[key], cached=True)
    timings = []

    def time_rule(a128, a64, a32):
        dec.set_batched_config(a128, a64, a32)
        dec.solve_batched(Y, eps, max_iters, want_r=False)  # warm-up
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            dec.solve_batched(Y, eps, max_iters, want_r=False)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        timings.append(dict(atoms128_above=a128, atoms64_above=a64, atoms32_above=a32,
                            ms=round(best * 1e3, 3)))
        if log:
            log(f"[tune] batched tiles: 128 above {a128}, 64 above {a64}, 32 above {a32}: "
                f"{best * 1e3:.2f} ms")

    for rule in (rules if rules is not None else batched_rules()):
        time_rule(*rule)
    if rules is None:
        w = min(timings, key=lambda d: d["ms"])
        for a32 in ATOMS32_ABOVE:
            time_rule(w["atoms128_above"], w["atoms64_above"], a32)
    win = min(timings, key=lambda d: d["ms"])
    cfg = dict(atoms128_above=win["atoms128_above"], atoms64_above=win["atoms64_above"],
               atoms32_above=win["atoms32_above"])
    dec.set_batched_config(**cfg)
    entry = dict(config=cfg, ms=win["ms"], timings=timings)
    if use_cache:
        cache[key] = entry
        _store_cache(cache)
    return dict(entry, cached=False)
