#!/usr/bin/env python3
"""Benchmark of the Matching Pursuit decoder on one MI355X.

A step is one whole decode (Section 3 loop until ||r|| <= eps ||y|| or T
steps) of one synthetic signal through the C ABI (mp_solve), with the
dictionary and y already resident in HBM.  Default workload: N=8192,
M=32768 (1 GiB FP32 dictionary), K=512, eps=1e-5, T=20K.

Prints ONE JSON line.  `value` is MP iterations per second over the timed
steps; `roofline` is the correlation kernel's algorithmic HBM bandwidth
(dictionary + residual bytes per launch / mean launch time from HIP events on
the decode stream) against the 8 TB/s peak and against the read rate a plain
streaming kernel reaches on the same device; `cpu_baseline` is the FP64
oracle timed on a bounded sample of the same decode on this host, on every
core and on one.  The line also carries the reduced-precision forms (BF16 and
FP8 dictionaries, both value laws, N=8192, M=32768, K=256), the small
single-signal workloads (N=256 and N=2048, cache-resident), the batched form,
the ragged instances (FP32 and BF16), the FP64 decode and the OMP decode of
the same workload, the decode on the sign-bit Bernoulli dictionary of the
same sizes, and the Fig. 1 error grid (each skippable, see --help).

Errors per result: after the GPU legs, the oracle checks what each leg
decoded (untimed): every step of a single-signal decode is judged against
the FP64 correlations of the decode's own state (selections that differ from
the FP64 argmax where the top-two gap exceeds 1e-5 ||r|| are counted as
misses; for the reduced-precision forms these are re-scoring misses), the
oracle replays the decode's atoms in FP64 and x~ and r are compared with the
replay, and the index sequence is compared with the oracle's own free run
over a sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MP iters/s & achieved HBM GB/s (1 signal); signals/s batched BF16 vs FP32"
HBM_PEAK_GBS = 8000.0
# counter-derived HBM traffic of each single-signal step kernel, and every
# source file that kernel is compiled from (the record is used only while
# those sources are unchanged)
_CSRC = os.path.join(ROOT, "paper_0809_1833_amd", "csrc")
TRAFFIC = {
    "f32": (os.path.join(ROOT, "profiles", "mp_step_f32_traffic.json"),
            [os.path.join(_CSRC, f) for f in ("k_f32.hip", "k_common.h", "mp_internal.h")]),
    "bf16": (os.path.join(ROOT, "profiles", "mp_step_lp_bf16_traffic.json"),
             [os.path.join(_CSRC, f) for f in ("k_lowp.hip", "k_lowp.h", "k_common.h",
                                               "mp_internal.h")]),
    "fp8": (os.path.join(ROOT, "profiles", "mp_step_lp_fp8_traffic.json"),
            [os.path.join(_CSRC, f) for f in ("k_lowp.hip", "k_lowp.h", "k_common.h",
                                              "mp_internal.h")]),
    "f64": (os.path.join(ROOT, "profiles", "mp_step_f64_traffic.json"),
            [os.path.join(_CSRC, f) for f in ("k_f64.hip", "k_common.h", "k_key2.h",
                                              "mp_internal.h")]),
    "sign": (os.path.join(ROOT, "profiles", "mp_step_sign_traffic.json"),
             [os.path.join(_CSRC, f) for f in ("k_sign.hip", "k_common.h", "k_key2.h",
                                               "mp_internal.h")]),
    "omp": (os.path.join(ROOT, "profiles", "omp_select_traffic.json"),
            [os.path.join(_CSRC, f) for f in ("k_omp.hip", "k_common.h", "mp_internal.h")]),
    # ragged solves: bytes per solve of the 512-instance workload (n = m = 0)
    "ragged_f32": (os.path.join(ROOT, "profiles", "ragged_f32_traffic.json"),
                   [os.path.join(_CSRC, f) for f in ("k_ragged.hip", "k_common.h", "k_lowp.h",
                                                     "mp_internal.h")]),
    "ragged_bf16": (os.path.join(ROOT, "profiles", "ragged_bf16_traffic.json"),
                    [os.path.join(_CSRC, f) for f in ("k_ragged.hip", "k_common.h", "k_lowp.h",
                                                      "mp_internal.h")]),
}
ESIZE = {"f64": 8.0, "f32": 4.0, "bf16": 2.0, "fp8": 1.0}
KERNEL = {"f64": "k_mp_step_f64", "f32": "k_mp_step_f32", "bf16": "k_mp_step_lp",
          "fp8": "k_mp_step_lp"}

WORKLOADS = {
    "c1b": "N=8192, M=32768 (FP32 dictionary 1 GiB), K=512, eps=1e-5, T=10240, single signal",
    "c1a": "N=2048, M=8192 (FP32 dictionary 64 MiB), K=128, eps=1e-5, T=2560, single signal",
    "c0": "N=256, M=1024, K=10, eps=1e-6, T=2000, single signal",
    "c2": "N=8192, M=32768, K=256, eps=1e-5, T=5120, single signal, reduced-precision dictionary "
          "with FP32 re-scoring of the 8 best candidates",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash(storage="f32"):
    h = hashlib.sha256()
    for path in TRAFFIC[storage][1]:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(n, m, storage="f32"):
    """HBM bytes per step launch from committed rocprofv3 counter runs, or
    None when absent, for another size, or taken on a different kernel source."""
    try:
        with open(TRAFFIC[storage][0]) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_hash(storage) or d.get("n") != n or d.get("m") != m:
        return None
    return d.get("bytes_per_launch")


def step_bytes(n, m, storage):
    """Algorithmic bytes of one iteration's launch: the dictionary copy once,
    r once, and for the reduced-precision forms the FP8 scales and the 8 FP32
    candidate columns re-scored."""
    rsize = 8.0 if storage == "f64" else 4.0
    b = ESIZE[storage] * n * m + rsize * n
    if storage == "fp8":
        b += 4.0 * m
    if storage in ("bf16", "fp8"):
        b += 8 * 4.0 * n
    return b


def time_decodes(dec, y, p, steps, warmup, profile_every, x, r, stream=None, omp=False,
                 **solve_kw):
    """Warm up, then time `steps` whole decodes; the step kernel's launches are
    timed with HIP events on the decode stream, over windows of profile_every
    consecutive launches (OMP: every profile_every-th selection launch).
    ``omp``: decode with Orthogonal Matching Pursuit (the selection pass is
    the timed kernel)."""
    import torch
    for _ in range(warmup):
        dec.solve(y, p.eps, p.max_iters, x=x, r=r, omp=omp, **solve_kw)
    dec.set_profiling(profile_every)
    torch.cuda.synchronize()
    iters, kt_ms, kt_n, stops = 0, 0.0, 0, set()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = dec.solve(y, p.eps, p.max_iters, x=x, r=r, stream=stream, omp=omp, **solve_kw)
        iters += out["iters"]
        if out.get("persistent"):
            stops.add("persistent")
        ms, cnt = dec.kernel_time()
        kt_ms += ms * cnt
        kt_n += cnt
        stops.add(out["stop"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dec.set_profiling(0)
    return iters, dt, kt_ms / max(kt_n, 1), kt_n, stops


def bench_f64(seed: int, steps: int = 2, warmup: int = 1, profile_every: int = 16):
    """FP64 decode of the same N=8192, M=32768 workload (2 GiB FP64
    dictionary): iters/s and the step kernel's algorithmic HBM bandwidth."""
    import numpy as np
    import torch

    import mpgen
    from paper_0809_1833_amd.mp import Decoder

    p = mpgen.make_problem("c1b", seed, precision="f64")
    n, m = p.n, p.m
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(p.y).cuda()
    del p.psi
    with Decoder(psi, storage="f64") as dec:
        del psi
        x = torch.empty(m, dtype=torch.float64, device="cuda")
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        iters, dt, avg_ms, kt_n, stops = time_decodes(dec, y, p, steps, warmup, profile_every,
                                                      x, r)
    b = step_bytes(n, m, "f64")
    achieved = b / (avg_ms * 1e-3) / 1e9 if kt_n else None
    return {"workload": f"N={n}, M={m} (FP64 dictionary 2 GiB), K=512, eps=1e-5, T=10240, "
                        "single signal, FP64 throughout",
            "iters_per_s": round(iters / dt, 3), "ms_per_decode": round(dt / steps * 1e3, 3),
            "iters_per_decode": iters // max(steps, 1), "stop": sorted(stops),
            "roofline": {"bound": "hbm", "kernel": KERNEL["f64"],
                         "achieved": round(achieved, 2) if achieved else None,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                         "traffic": traffic_from_counters(n, m, "f64"),
                         "bytes_per_launch": b, "avg_launch_us": round(avg_ms * 1e3, 3),
                         "launches": kt_n}}


def sign_step_bytes(n, m):
    """Algorithmic bytes of one sign-bit launch: every column's bits once,
    its FP64 correlation read and written, and r's rows in FP64 (read and
    written) and FP32 (written)."""
    return n * m / 8.0 + 16.0 * m + 20.0 * n


# LDS bandwidth of the chip: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4


def bench_sign(seed: int, steps: int = 3, warmup: int = 1, profile_every: int = 16,
               max_iters=None):
    """Decode on the Bernoulli dictionary of eq. 13 held as sign bits
    (mp_create_signs): N=8192, M=32768 (32 MiB of bits), K=512, eps=1e-5,
    T=10240.  The correlations are carried by exact Gram updates (XOR and
    bit count).  Where the decode runs as one persistent launch with the bits
    held in LDS, its roofline is the time per step (bound by the exchange of
    the workgroups' records) with the LDS rate of the bits beside it; the
    same decode with one launch per step is timed too, each launch streaming
    the bits once from HBM (algorithmic bytes per launch over its mean launch
    time)."""
    import torch

    import mpgen
    from paper_0809_1833_amd.mp import Decoder

    p = mpgen.make_sign_problem("c1b", seed)
    if max_iters is not None:
        p.max_iters = min(p.max_iters, max_iters)
    n, m = p.n, p.m
    bits = torch.from_numpy(p.bits.view("int32")).cuda()
    y = torch.from_numpy(p.y).cuda()
    with Decoder(bits, storage="sign", n=n) as dec:
        del bits
        x = torch.empty(m, dtype=torch.float32, device="cuda")
        r = torch.empty(n, dtype=torch.float32, device="cuda")
        iters, dt, avg_ms, kt_n, stops = time_decodes(dec, y, p, steps, warmup, profile_every,
                                                      x, r)
        # the same decode with one launch per step, for comparison
        s_it, s_dt, s_ms, s_n, s_stops = time_decodes(dec, y, p, steps, warmup, profile_every,
                                                      x, r, step_launches=True)
    persistent = "persistent" in stops
    stops.discard("persistent")
    bits = n * m / 8.0
    b = sign_step_bytes(n, m)
    s_ach = b / (s_ms * 1e-3) / 1e9 if s_n else None
    lds = bits / (avg_ms * 1e-3) / 1e9 if kt_n else None
    step = {"bound": "hbm", "kernel": "k_mp_step_sign",
            "iters_per_s": round(s_it / s_dt, 3),
            "achieved": round(s_ach, 2) if s_ach else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(s_ach / HBM_PEAK_GBS, 4) if s_ach else None,
            "traffic": traffic_from_counters(n, m, "sign"), "bytes_per_launch": b,
            "avg_launch_us": round(s_ms * 1e3, 3), "launches": s_n}
    out = {"workload": f"N={n}, M={m}, Bernoulli dictionary (eq. 13) as sign bits "
                       "(32 MiB), K=512, eps=1e-5, T=10240, single signal",
           "iters_per_s": round(iters / dt, 3), "ms_per_decode": round(dt / steps * 1e3, 3),
           "iters_per_decode": iters // max(steps, 1), "stop": sorted(stops),
           "persistent": persistent}
    if persistent:
        # the bits stay in LDS for the whole decode: a step reads them from
        # LDS, and waits for every workgroup's record of the step before
        out["roofline"] = {"bound": "exchange", "kernel": "k_sign_persist",
                           "avg_step_us": round(avg_ms * 1e3, 3), "steps": kt_n,
                           "lds": {"achieved": round(lds, 2) if lds else None,
                                   "peak": LDS_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(lds / LDS_PEAK_GBS, 4) if lds else None,
                                   "bytes_per_step": bits}}
        out["step_launches"] = step
    else:
        out["roofline"] = step
    return out


def bench_phase(seed: int):
    """The Fig. 1 experiment on the batched decoder: M=1000, a 20 x 20 grid of
    sigma = K/M and rho = N/M (steps of 0.05), 100 trials per cell over 4
    Bernoulli dictionaries per rho, eps=1e-7, T=N.  Reports decodes per second
    of device time and a few landmarks of E(sigma, rho)."""
    from paper_0809_1833_amd import phase
    res = phase.phase_diagram(seed=seed, log=log)
    E = res["E"]
    return {"workload": "Fig. 1 grid: M=1000, sigma, rho in {0.05..1.0} (20 x 20), 100 trials "
                        "per cell, Bernoulli dictionary, U[-1,1] nonzeros, eps=1e-7, T=N",
            "decodes": res["decodes"], "decode_s": round(res["decode_seconds"], 3),
            "signals_per_s": round(res["signals_per_s"], 1),
            "E_percent": {"sigma0.05_rho1.0": round(float(E[-1][0]), 6),
                          "sigma0.25_rho0.5": round(float(E[9][4]), 4),
                          "sigma0.5_rho0.5": round(float(E[9][9]), 4),
                          "sigma1.0_rho0.05": round(float(E[0][-1]), 4)}}


def host_cpu():
    """(CPU model name, cores this process may run on) of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def stream_ceiling():
    """Read rate (GB/s) of a plain streaming kernel on this device: the probe
    built beside the library, each workgroup reading one contiguous chunk of a
    1 GiB buffer with 16-byte non-temporal loads (mean of 10 launches, HIP
    events).  None when the probe is not built or fails."""
    exe = os.path.join(ROOT, "paper_0809_1833_amd", "probe", "stream_probe")
    if not os.path.exists(exe):
        return None
    try:
        out = subprocess.run([exe, "chunk", "1024", "10"], capture_output=True, text=True,
                             timeout=120)
    except (OSError, subprocess.TimeoutExpired):
        return None
    if out.returncode != 0:
        return None
    for line in out.stdout.splitlines():
        try:
            return float(json.loads(line)["gbps"])
        except (ValueError, KeyError):
            continue
    return None


def hbm_roofline(kernel, bytes_per_launch, avg_ms, launches, traffic=None, ceiling=None,
                 bound="hbm"):
    """Roofline record of a streaming kernel: algorithmic bytes per launch over
    its mean launch time, against the 8 TB/s peak and the streaming probe's
    measured ceiling."""
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if launches else None
    d = {"bound": bound, "kernel": kernel,
         "achieved": round(achieved, 2) if achieved else None,
         "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
         "traffic": traffic, "bytes_per_launch": bytes_per_launch,
         "avg_launch_us": round(avg_ms * 1e3, 3), "launches": launches}
    if ceiling and achieved:
        d["stream_ceiling_gbps"] = round(ceiling, 1)
        d["frac_of_stream_ceiling"] = round(achieved / ceiling, 4)
    return d


def traced_decode(dec, y, p, **kw):
    """One untimed decode with its whole per-step record (atoms, coefficients,
    the residual after every step), as numpy arrays for the oracle's checks."""
    import torch
    out = dec.solve(y, p.eps, p.max_iters, trace_cap=max(p.max_iters, 1), trace_r=True, **kw)
    torch.cuda.synchronize()
    g = {"iters": out["iters"], "stop": out["stop"], "yy": out["yy"], "rr": out["rr"]}
    for k in ("x", "r", "idx", "coef", "r_trace"):
        g[k] = out[k].cpu().numpy() if k in out else None
    return g


def concurrent_decodes(psi, y, p, storage, steps, nd=4):
    """Stream-ordered decodes of the same signal on `nd` contexts, one stream
    each: every round issues one decode per context, then collects them all.
    Returns the aggregate iterations/s."""
    import torch

    from paper_0809_1833_amd.mp import Decoder

    decs = [Decoder(psi, storage=storage) for _ in range(nd)]
    streams = [torch.cuda.Stream() for _ in range(nd)]
    xs = [torch.empty(p.m, dtype=torch.float32, device="cuda") for _ in range(nd)]
    rs = [torch.empty(p.n, dtype=torch.float32, device="cuda") for _ in range(nd)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())

    def round_():
        for d, s, x, r in zip(decs, streams, xs, rs):
            d.solve(y, p.eps, p.max_iters, x=x, r=r, stream=s, asynchronous=True)
        return sum(d.result()["iters"] for d in decs)

    try:
        round_()
        torch.cuda.synchronize()
        total = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            total += round_()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        for d in decs:
            d.close()
    return {"contexts": nd, "streams": nd, "decodes": nd * steps,
            "iters_per_s": round(total / dt, 3)}


def bench_single(p, storage, steps, warmup, profile_every, ceiling, workload, rescore_k=0,
                 check=True):
    """Time `steps` decodes of problem p with the given dictionary storage,
    then (``check``) decode it once more with the whole per-step record.
    Returns (the leg's record, the decode to check against the oracle or
    None)."""
    import torch

    from paper_0809_1833_amd.mp import Decoder

    n, m = p.n, p.m
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(p.y).cuda()
    with Decoder(psi, storage=storage) as dec:
        x = torch.empty(m, dtype=torch.float32, device="cuda")
        r = torch.empty(n, dtype=torch.float32, device="cuda")
        iters, dt, avg_ms, kt_n, stops = time_decodes(dec, y, p, steps, warmup, profile_every,
                                                      x, r, rescore_k=rescore_k)
        g = traced_decode(dec, y, p, rescore_k=rescore_k) if check else None
        one_launch = "persistent" in stops
        stops.discard("persistent")
        conc = None
        if one_launch:
            # the same decode with one launch per step, for comparison
            s_it, s_dt, s_ms, s_n, _ = time_decodes(dec, y, p, steps, warmup, profile_every,
                                                    x, r, rescore_k=rescore_k,
                                                    step_launches=True)
            conc = concurrent_decodes(psi, y, p, storage, steps)
        del psi
    leg = {"workload": workload, "storage": storage,
           "iters_per_s": round(iters / dt, 3), "ms_per_decode": round(dt / steps * 1e3, 3),
           "us_per_iter": round(dt / max(iters, 1) * 1e6, 3),
           "iters_per_decode": iters // max(steps, 1), "stop": sorted(stops),
           "one_launch": one_launch}
    b = step_bytes(n, m, storage)
    if one_launch:
        # the whole decode in one launch with the dictionary's shares in LDS:
        # the time per step, the dictionary bytes per step read from LDS
        leg["roofline"] = {"bound": "exchange", "kernel": "k_f32_small",
                           "avg_step_us": round(avg_ms * 1e3, 3), "steps": kt_n,
                           "lds_bytes_per_step": 4.0 * n * m}
        leg["step_launches"] = {
            "iters_per_s": round(s_it / s_dt, 3), "us_per_iter": round(s_dt / max(s_it, 1) * 1e6, 3),
            "roofline": hbm_roofline(KERNEL[storage], b, s_ms, s_n,
                                     traffic_from_counters(n, m, storage), ceiling)}
        leg["one_launch_over_step_launches"] = round((iters / dt) / (s_it / s_dt), 3)
        conc["over_one_stream"] = round(conc["iters_per_s"] / (iters / dt), 3)
        leg["concurrent"] = conc
    else:
        leg["roofline"] = hbm_roofline(KERNEL[storage], b, avg_ms, kt_n,
                                       traffic_from_counters(n, m, storage), ceiling)
    return leg, g


# ---- the oracle's side: baseline timing and the checks of each decode -------

def cpu_baseline(p, budget_s=12.0, one_thread_s=6.0):
    """The FP64 oracle on a bounded sample of the same decode: its first
    iterations on every core, then on one thread.  Returns (the record, the
    all-core run, whose index sequence the decode is compared with)."""
    import oracle
    solve = oracle.solve64 if p.psi.dtype.itemsize == 8 else oracle.solve
    model, avail = host_cpu()
    threads = oracle.num_threads()

    def sample(budget):
        t0 = time.perf_counter()
        solve(p.psi, p.y, p.eps, 2, trace=True)
        per = max((time.perf_counter() - t0) / 2.0, 1e-6)
        iters = int(max(3, min(p.max_iters, budget / per)))
        t0 = time.perf_counter()
        res = solve(p.psi, p.y, p.eps, iters, trace=True)
        return res, time.perf_counter() - t0

    res, dt = sample(budget_s)
    oracle.set_num_threads(1)
    try:
        res1, dt1 = sample(one_thread_s)
    finally:
        oracle.set_num_threads(threads)
    rec = dict(value=round(res.iters / dt, 3), unit="iters/s", cores=threads, kind="oracle",
               sample=f"first {res.iters} MP iterations of the same decode (FP64 correlations, "
                      f"{dt:.1f} s, per-step trace kept)",
               cpu_model=model, host_cores=avail,
               one_thread={"value": round(res1.iters / dt1, 3), "unit": "iters/s", "cores": 1,
                           "sample": f"first {res1.iters} iterations ({dt1:.1f} s)"})
    return rec, res


def _states(yv, rtrace, a, b):
    """The decode's states before steps a..b-1 as an (N, b-a) FP64 matrix."""
    return np.stack([yv if t == 0 else rtrace[t - 1] for t in range(a, b)],
                    axis=1).astype(np.float64)


def oracle_errors(psi, y, g, free=None, y64=False, tol_sel=1e-5, local=True, chunk=512,
                  corr=None):
    """Errors of one single-signal decode ``g`` (from traced_decode) against
    the FP64 oracle:
      * every step's selection against the FP64 argmax of the decode's own
        state (misses: a different atom where the top-two gap exceeds
        tol_sel ||r_t||; near_ties: a different atom at a smaller gap);
      * x~ and r against the oracle replaying the decode's atoms in FP64
        (x~ relative to ||x~||, r relative to ||y||), and y - Psi x~ - r;
      * with ``free`` (the oracle's own run over a sample), the number of
        leading steps whose atoms agree.
    ``corr``: an ``oracle.Correlator`` of psi to reuse."""
    import oracle
    T = int(g["iters"])
    idx = np.asarray(g["idx"], dtype=np.int64)[:T]
    yv = np.asarray(y, dtype=np.float64) if y64 else np.asarray(y, np.float32).astype(np.float64)
    ynorm = float(np.linalg.norm(yv))
    out = {"iters": T, "stop": g["stop"],
           "final_r_over_y": float(np.sqrt(max(g["rr"], 0.0) / g["yy"])) if g["yy"] else 0.0}
    if local and T and g.get("r_trace") is not None:
        corr = oracle.Correlator(psi) if corr is None else corr
        exact = misses = ties = 0
        for a in range(0, T, chunk):
            b = min(T, a + chunk)
            R = _states(yv, g["r_trace"], a, b)
            best, _, gap = oracle.top_gap(corr.many(R))
            ex = gap > tol_sel * np.linalg.norm(R, axis=0)
            differ = idx[a:b] != best
            exact += int(ex.sum())
            misses += int((differ & ex).sum())
            ties += int((differ & ~ex).sum())
        out.update(steps_judged=T, gap_decided_steps=exact, misses=misses, near_ties=ties)
    if T:
        rep = oracle.replay(psi, yv if y64 else np.asarray(y, np.float32), idx.astype(np.int32),
                            check_ties=False, y64=y64)
        xg = np.asarray(g["x"], np.float64)
        rg = np.asarray(g["r"], np.float64)
        out["x_rel_err_vs_replay"] = float(np.linalg.norm(xg - rep.x) /
                                           max(np.linalg.norm(rep.x), 1e-300))
        out["r_err_vs_replay_over_y"] = float(np.linalg.norm(rg - rep.r) / max(ynorm, 1e-300))
        nz = np.flatnonzero(xg)
        cols = np.asarray(psi[:, nz], dtype=np.float64)
        out["defect_over_y"] = float(np.linalg.norm(yv - cols @ xg[nz] - rg) / max(ynorm, 1e-300))
    if free is not None:
        k = min(len(free.idx), T)
        mism = np.flatnonzero(np.asarray(free.idx[:k], np.int64) != idx[:k])
        out["index_match_steps"] = int(mism[0]) if mism.size else int(k)
        out["index_compared_steps"] = int(k)
    return out


def _round_errors(d):
    return {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in d.items()}


def bench_batched(seed: int, reps: int = 3, warmup: int = 1, sequential: bool = True,
                  check: bool = True):
    """Batched workload: 256 signals, K_b ~ U{16..256}, sharing one N=2048,
    M=8192 dictionary.  signals/s of mp_solve_batched (BF16 matrix-core
    correlations, FP32 re-scoring) and, for comparison, of FP32 mp_solve run
    signal after signal on the same inputs; MFMA utilisation of the product
    kernel = 2 N M (sum of per-signal iterations) / (its summed launch time).
    Returns (the record, the traced decode for the oracle's checks)."""
    import torch

    import mpgen
    from paper_0809_1833_amd import tune
    from paper_0809_1833_amd.mp import Decoder

    bt = mpgen.make_batch(seed)
    n, m, nb = bt.psi.shape[0], bt.psi.shape[1], bt.y.shape[1]
    psi = torch.from_numpy(np.ascontiguousarray(bt.psi.T)).cuda().t()
    Y = torch.from_numpy(np.ascontiguousarray(bt.y.T)).cuda().t()
    caps = [int(v) for v in bt.max_iters]
    out = {"workload": f"N={n}, M={m}, B={nb} signals, K_b ~ U{{16..256}}, eps={bt.eps}, "
                       "T_b=20 K_b, shared dictionary"}
    with Decoder(psi, storage="bf16") as dec:
        # the product's tile rule, from the tuner's cache or timed here
        tn = tune.tune_batched(dec, Y, bt.eps, caps, reps=2, log=log)
        out["config"] = tn["config"]
        out["tuned_from_cache"] = tn["cached"]
        if not tn["cached"]:
            out["tile_rule_ms"] = {
                f"{d['atoms128_above']}/{d['atoms64_above']}/{d['atoms32_above']}": d["ms"]
                for d in tn["timings"]}
        for _ in range(warmup):
            dec.solve_batched(Y, bt.eps, caps, want_r=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = dec.solve_batched(Y, bt.eps, caps, want_r=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        total_iters = sum(res["iters"])
        out.update(signals_per_s_bf16_batched=round(nb / dt, 2), batch_ms=round(dt * 1e3, 3),
                   total_iters=total_iters, max_iters=max(res["iters"]),
                   stops=sorted(set(res["stop"])))
        dec.set_profiling(1)
        dec.solve_batched(Y, bt.eps, caps, want_r=False)
        ms, cnt = dec.kernel_time()
        dec.set_profiling(0)
        flops = 2.0 * n * m * total_iters
        gemm_s = ms * cnt * 1e-3
        out["mfma"] = {"bound": "mfma", "kernel": "k_bcorr", "achieved": round(flops / gemm_s / 1e12, 2),
                       "peak": 2500.0, "unit": "TFLOP/s",
                       "frac": round(flops / gemm_s / 1e12 / 2500.0, 4),
                       "rounds": cnt, "gemm_ms_per_batch": round(ms * cnt, 3)}
        # the same products against memory: every round reads the BF16
        # dictionary once and each active signal's BF16 residual once (below
        # the BF16 ridge of about 312 flop/B even at 256 signals)
        opnd = cnt * 2.0 * n * m + 2.0 * n * total_iters
        out["operand_bytes"] = {"bound": "hbm", "kernel": "k_bcorr",
                                "achieved": round(opnd / gemm_s / 1e9, 2), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(opnd / gemm_s / 1e9 / HBM_PEAK_GBS, 4),
                                "bytes_per_batch": opnd,
                                "flop_per_byte": round(flops / opnd, 1)}
        # one more decode with every signal's atoms recorded, for the checks
        g = None
        if check:
            tr = dec.solve_batched(Y, bt.eps, caps, trace_cap=max(max(caps), 1))
            torch.cuda.synchronize()
            g = {"iters": tr["iters"], "stop": tr["stop"], "rr": tr["rr"], "yy": tr["yy"],
                 "idx": tr["idx"].cpu().numpy(), "x": tr["x"].cpu().numpy(),
                 "r": tr["r"].cpu().numpy()}
    if sequential:
        with Decoder(psi, storage="f32") as dec:
            x = torch.empty(m, dtype=torch.float32, device="cuda")
            r = torch.empty(n, dtype=torch.float32, device="cuda")
            ys = [Y[:, b].contiguous() for b in range(nb)]
            dec.solve(ys[0], bt.eps, caps[0], x=x, r=r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for b in range(nb):
                dec.solve(ys[b], bt.eps, caps[b], x=x, r=r)
            torch.cuda.synchronize()
            dts = time.perf_counter() - t0
        out["signals_per_s_f32_sequential"] = round(nb / dts, 2)
        out["batched_over_sequential"] = round(dts / dt, 2)
    return out, {"psis": [bt.psi], "ys": [bt.y[:, b] for b in range(nb)], "eps": bt.eps,
                 "dict_of": [0] * nb, "g": g}


def bench_ragged(seed: int, storages=("f32", "bf16"), reps: int = 3, tune_reps: int = 2,
                 check: bool = True):
    """Ragged workload: 512 independent problems, N_i ~ U{128,256,512,1024},
    M_i = 4 N_i, K_i = N_i / 16, eps = 1e-5, T_i = 20 K_i, each with its own
    dictionary, decoded in one persistent graph-replayed launch whose shape
    the autotuner picks, once per dictionary storage.  Reports problems/s and
    the aggregate algorithmic dictionary bandwidth sum_i iters_i * bytes(Psi_i)
    / time.  Returns ({storage: record}, {storage: decode to check})."""
    import torch

    import mpgen
    from paper_0809_1833_amd import tune
    from paper_0809_1833_amd.mp import RaggedDecoder

    probs = mpgen.make_ragged(seed)
    caps = [p.max_iters for p in probs]
    psis = [torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t() for p in probs]
    yp = torch.from_numpy(np.concatenate([p.y for p in probs]).astype(np.float32)).cuda()
    recs, checks = {}, {}
    for storage in storages:
        esize = 4.0 if storage == "f32" else 2.0
        out = {"workload": "512 instances, N_i ~ U{128,256,512,1024}, M_i = 4 N_i, K_i = N_i/16, "
                           f"eps=1e-5, T_i = 20 K_i, own dictionary each, {storage} storage"}
        with RaggedDecoder(psis, storage=storage) as dec:
            tuned = tune.tune_ragged(dec, yp, 1e-5, caps, reps=tune_reps, log=log)
            x = torch.empty(dec.x_off[-1], dtype=torch.float32, device="cuda")
            dec.solve(yp, 1e-5, caps, want_r=False, x_out=x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                res = dec.solve(yp, 1e-5, caps, want_r=False, x_out=x)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            dec.set_profiling(1)
            dec.solve(yp, 1e-5, caps, want_r=False, x_out=x)
            kms, _ = dec.kernel_time()
            dec.set_profiling(0)
            g = None
            if check:
                tr = dec.solve(yp, 1e-5, caps, trace_cap=max(caps))
                torch.cuda.synchronize()
                xo, yo = dec.x_off, dec.y_off
                xs, rs = tr["x"].cpu().numpy(), tr["r"].cpu().numpy()
                ti = tr["idx"].cpu().numpy()
                g = {"iters": tr["iters"], "stop": tr["stop"], "rr": tr["rr"], "yy": tr["yy"],
                     "idx": ti, "x": [xs[xo[i]:xo[i + 1]] for i in range(len(probs))],
                     "r": [rs[yo[i]:yo[i + 1]] for i in range(len(probs))]}
        nbytes = sum(it * esize * p.n * p.m for it, p in zip(res["iters"], probs))
        achieved = nbytes / (kms * 1e-3) / 1e9
        out.update(problems_per_s=round(len(probs) / dt, 2), solve_ms=round(dt * 1e3, 3),
                   total_iters=sum(res["iters"]), stops=sorted(set(res["stop"])),
                   config=tuned["config"], tuned_from_cache=tuned["cached"],
                   roofline={"bound": "hbm", "kernel": "k_ragged", "achieved": round(achieved, 2),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "traffic": traffic_from_counters(0, 0, "ragged_" + storage),
                             "bytes_per_solve": nbytes,
                             "launch_ms": round(kms, 3),
                             "note": "algorithmic bytes count every instance's dictionary "
                                     "once per iteration; the counters (traffic, bytes per "
                                     "solve) show the dictionaries read from memory each "
                                     "time, none re-read from L2"})
        recs[storage] = out
        checks[storage] = {"psis": [p.psi for p in probs], "ys": [p.y for p in probs],
                           "eps": 1e-5, "dict_of": list(range(len(probs))), "g": g}
    return recs, checks


def many_errors(chk, free_every=8, free_cap=400):
    """Per-signal errors of a batched or ragged decode against the FP64
    oracle: x~ and r against the oracle replaying each signal's atoms, the
    final ||r||/||y||, and, for every ``free_every``-th signal, the leading
    steps (of at most ``free_cap``) whose atoms agree with the oracle's own
    run."""
    import oracle
    g = chk["g"]
    xe, re_, fr, match, compared = [], [], [], [], []
    for b, (yb, d) in enumerate(zip(chk["ys"], chk["dict_of"])):
        psi = chk["psis"][d]
        T = int(g["iters"][b])
        idx = np.asarray(g["idx"][b][:T], dtype=np.int32)
        xg = np.asarray(g["x"][b] if isinstance(g["x"], list) else g["x"][:, b], np.float64)
        rg = np.asarray(g["r"][b] if isinstance(g["r"], list) else g["r"][:, b], np.float64)
        yv = np.asarray(yb, np.float32).astype(np.float64)
        ynorm = float(np.linalg.norm(yv))
        if T:
            rep = oracle.replay(psi, np.asarray(yb, np.float32), idx, check_ties=False)
            xe.append(float(np.linalg.norm(xg - rep.x) / max(np.linalg.norm(rep.x), 1e-300)))
            re_.append(float(np.linalg.norm(rg - rep.r) / max(ynorm, 1e-300)))
        fr.append(float(np.sqrt(max(g["rr"][b], 0.0) / g["yy"][b])) if g["yy"][b] else 0.0)
        if b % free_every == 0:
            free = oracle.solve(psi, np.asarray(yb, np.float32), chk["eps"], min(free_cap, T))
            k = min(free.iters, T)
            mism = np.flatnonzero(free.idx[:k].astype(np.int64) != idx[:k])
            match.append(int(mism[0]) if mism.size else int(k))
            compared.append(int(k))
    return {"signals": len(chk["ys"]),
            "x_rel_err_vs_replay_max": max(xe, default=0.0),
            "x_rel_err_vs_replay_median": float(np.median(xe)) if xe else 0.0,
            "r_err_vs_replay_over_y_max": max(re_, default=0.0),
            "final_r_over_y_max": max(fr, default=0.0),
            "index_match": {"signals": len(match), "steps_matched": int(sum(match)),
                            "steps_compared": int(sum(compared)),
                            "signals_fully_matched": int(sum(a == c for a, c in
                                                             zip(match, compared)))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1b", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "fp8", "f64"],
                    help="dictionary copy the correlation pass streams (f64: the FP64 "
                         "decode, FP64 inputs)")
    ap.add_argument("--dist", default="normal", choices=["normal", "loguniform"])
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the streaming probe run that gives the measured read ceiling")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle: no CPU baseline and no error checks")
    ap.add_argument("--no-reduced", action="store_true",
                    help="skip the BF16 / FP8 dictionary legs (N=8192, M=32768, K=256)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the N=256 and N=2048 single-signal legs")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form measurement added to the line")
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the ragged-instances measurement added to the line")
    ap.add_argument("--no-f64", action="store_true",
                    help="skip the FP64-decode measurement added to the line")
    ap.add_argument("--no-sign", action="store_true",
                    help="skip the sign-bit Bernoulli decode")
    ap.add_argument("--no-omp", action="store_true",
                    help="skip the Orthogonal Matching Pursuit decode added to the line")
    ap.add_argument("--no-phase", action="store_true",
                    help="skip the Fig. 1 experiment (reconstruction error grid) added to the line")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched leg: skip the FP32 comparison that decodes the same signals "
                         "one by one")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="time the step kernel with HIP events over windows of k consecutive "
                         "launches (OMP: every k-th selection launch)")
    ap.add_argument("--max-iters", type=int, default=None,
                    help="cap each decode at this many iterations (short profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the decoder is built and measured on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    import mpgen
    from paper_0809_1833_amd.mp import Decoder

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ceiling = None if args.no_ceiling else stream_ceiling()
    log(f"[bench] streaming ceiling {ceiling} GB/s; generating {args.workload} seed {args.seed}")
    prec = "f64" if args.storage == "f64" else "f32"
    p = mpgen.make_problem(args.workload, args.seed, dist=args.dist, precision=prec)
    if args.max_iters is not None:
        p.max_iters = min(p.max_iters, args.max_iters)
    n, m = p.n, p.m
    tdt = torch.float64 if prec == "f64" else torch.float32
    psi = torch.from_numpy(np.ascontiguousarray(p.psi.T)).cuda().t()
    y = torch.from_numpy(p.y).cuda()
    stream = torch.cuda.current_stream()
    dec = Decoder(psi, storage=args.storage)
    del psi
    x = torch.empty(m, dtype=tdt, device="cuda")
    r = torch.empty(n, dtype=tdt, device="cuda")
    log(f"[bench] warmup, then timing {args.steps} decodes")
    iters, dt, avg_ms, kt_n, stops = time_decodes(dec, y, p, args.steps, args.warmup,
                                                  args.profile_every, x, r, stream)
    log(f"[bench] {iters} iterations in {dt:.3f} s")
    one_launch = "persistent" in stops
    stops.discard("persistent")
    # the same decode once more, untimed, with its whole per-step record (for
    # the oracle's checks at the end)
    check = not args.no_cpu_baseline
    main_g = traced_decode(dec, y, p) if check else None

    bytes_per_launch = step_bytes(n, m, args.storage)
    rsize = 8.0 if prec == "f64" else 4.0
    bytes_per_iter = bytes_per_launch + 2 * rsize * n  # + residual read and written by the update
    line = {
        "metric": METRIC,
        "value": round(iters / dt, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 storage, f32 accumulate",
                  "fp8": "fp8-e4m3 storage, f32 accumulate", "f64": "f64"}[args.storage],
        "data": "synthetic (seeded Gaussian unit-column dictionary, K-sparse N(0,1) signal)",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "storage": args.storage, "dist": args.dist,
                   "iters_per_decode": iters // max(args.steps, 1),
                   "stop": sorted(stops), "seed": args.seed,
                   "max_iters": p.max_iters},
        "effective_gbps_whole_step": round(iters * bytes_per_iter / dt / 1e9, 2),
        "roofline": hbm_roofline(KERNEL[args.storage], bytes_per_launch, avg_ms, kt_n,
                                 traffic_from_counters(n, m, args.storage), ceiling),
    }
    if one_launch:
        # a small dictionary decoded in one launch from its shares in LDS: the
        # time per step, bound by the exchange of the workgroups' best keys
        line["config"]["one_launch"] = True
        line["roofline"] = {"bound": "exchange", "kernel": "k_f32_small",
                            "avg_step_us": round(avg_ms * 1e3, 3), "steps": kt_n,
                            "lds_bytes_per_step": 4.0 * n * m}
    if not args.no_omp and args.storage == "f32":
        log("[bench] OMP decode of the same signal")
        o_it, o_dt, o_ms, o_n, o_stops = time_decodes(dec, y, p, args.steps, args.warmup,
                                                      args.profile_every, x, r, stream, omp=True)
        o_ach = bytes_per_launch / (o_ms * 1e-3) / 1e9 if o_n else None
        line["omp"] = {
            "workload": f"{args.workload}, Orthogonal Matching Pursuit (QR re-fit, CGS2)",
            "iters_per_s": round(o_it / o_dt, 3), "ms_per_decode": round(o_dt / args.steps * 1e3, 3),
            "iters_per_decode": o_it // max(args.steps, 1), "stop": sorted(o_stops),
            "select_kernel": {"kernel": "k_omp_select", "avg_launch_us": round(o_ms * 1e3, 3),
                              "achieved": round(o_ach, 2) if o_ach else None, "unit": "GB/s",
                              "frac": round(o_ach / HBM_PEAK_GBS, 4) if o_ach else None,
                              "traffic": traffic_from_counters(p.n, p.m, "omp")}}
    dec.close()
    del y, x, r
    torch.cuda.empty_cache()

    # decodes to check against the oracle at the end: (where in the line, problem, decode)
    singles = [(("errors",), p, main_g, prec == "f64")]
    default_main = args.workload == "c1b" and args.storage == "f32"
    if default_main and not args.no_reduced:
        line["reduced_precision"] = {}
        base = None
        for dist in ("normal", "loguniform"):
            log(f"[bench] reduced-precision dictionaries, {dist} values")
            q = mpgen.make_problem("c2", args.seed, dist=dist, psi=base)
            base = q.psi
            if args.max_iters is not None:
                q.max_iters = min(q.max_iters, args.max_iters)
            for storage in ("bf16", "fp8"):
                leg, g = bench_single(q, storage, args.steps, args.warmup, args.profile_every,
                                      ceiling, f"c2: {WORKLOADS['c2']}, {dist} values",
                                      check=check)
                key = f"{storage}_{dist}"
                line["reduced_precision"][key] = leg
                singles.append((("reduced_precision", key, "errors"), q, g, False))
        del base
    if default_main and not args.no_small:
        line["small"] = {}
        for wl, steps in (("c0", 20), ("c1a", 5)):
            log(f"[bench] small single-signal workload {wl}")
            q = mpgen.make_problem(wl, args.seed)
            if args.max_iters is not None:
                q.max_iters = min(q.max_iters, args.max_iters)
            leg, g = bench_single(q, "f32", steps, args.warmup, args.profile_every, ceiling,
                                  f"{wl}: {WORKLOADS[wl]}", check=check)
            roof = leg["step_launches"]["roofline"] if leg["one_launch"] else leg["roofline"]
            roof["bound"] = "cache-resident"
            roof["note"] = ("the dictionary (%.0f MiB) fits in the 256 MB MALL: the bytes are "
                            "algorithmic, not HBM traffic" % (4.0 * q.n * q.m / 2 ** 20))
            line["small"][wl] = leg
            singles.append((("small", wl, "errors"), q, g, False))
    many = []
    if not args.no_batched:
        log("[bench] batched form (256 signals, shared dictionary)")
        line["batched"], chk = bench_batched(args.seed, sequential=not args.no_sequential,
                                             check=check)
        many.append((("batched", "errors"), chk))
    if not args.no_ragged:
        log("[bench] ragged instances (512 problems of uneven size), FP32 and BF16")
        recs, chks = bench_ragged(args.seed, check=check)
        line["ragged"] = recs["f32"]
        line["ragged_bf16"] = recs["bf16"]
        many.append((("ragged", "errors"), chks["f32"]))
        many.append((("ragged_bf16", "errors"), chks["bf16"]))
    if not args.no_f64 and args.storage != "f64":
        log("[bench] FP64 decode of the same workload")
        line["f64"] = bench_f64(args.seed)
    if not args.no_sign:
        log("[bench] sign-bit Bernoulli dictionary (same sizes)")
        line["sign"] = bench_sign(args.seed, max_iters=args.max_iters)
    if not args.no_phase:
        log("[bench] Fig. 1 experiment (batched decodes over the sigma-rho grid)")
        line["phase"] = bench_phase(args.seed)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle), then the oracle's checks of each decode")
        import oracle
        line["cpu_baseline"], free = cpu_baseline(p)
        frees = {id(p): free}
        corr = (None, None)  # (dictionary, its Correlator), reused by consecutive checks
        for where, q, g, y64 in singles:
            if id(q) not in frees:  # the oracle's own run: whole, or its first 200 steps at N=8192
                cap = min(q.max_iters, 200) if q.n >= 8192 else q.max_iters
                frees[id(q)] = oracle.solve(q.psi, q.y, q.eps, cap)
            if corr[0] is not q.psi:
                corr = (None, None)
                corr = (q.psi, oracle.Correlator(q.psi))
            err = _round_errors(oracle_errors(q.psi, q.y, g, free=frees[id(q)], y64=y64,
                                              corr=corr[1]))
            err["tol"] = "misses must be 0; x~, r within 1e-5 (FP32) of the FP64 replay"
            _put(line, where, err)
            log(f"[bench] checked {'/'.join(where)}")
        corr = None
        for where, chk in many:
            _put(line, where, _round_errors(many_errors(chk)))
            log(f"[bench] checked {'/'.join(where)}")
    print(json.dumps(line), flush=True)


def _put(d, path, value):
    for k in path[:-1]:
        d = d.setdefault(k, {})
    d[path[-1]] = value


if __name__ == "__main__":
    main()
