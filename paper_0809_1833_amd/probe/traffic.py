"""Turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs into HBM bytes per launch.

Each counter is read in KiB per dispatch.  The scale factor of each counter
comes from the probe's copy kernel, whose bytes read and written are known
exactly: factor = known bytes / (counter KiB * 1024).  The result is written
as JSON (by default ``profiles/<kernel>_traffic.json``) together with the
SHA-256 prefix of the kernel's source files, so a benchmark can tell when the
kernel has changed since the counters were taken.

Usage (after the four counter runs described in the profile summaries):

    python -m paper_0809_1833_amd.probe.traffic --kernel k_mp_step_f32 \\
        --source paper_0809_1833_amd/csrc/k_f32.hip \\
        --source paper_0809_1833_amd/csrc/k_common.h \\
        --source paper_0809_1833_amd/csrc/mp_internal.h --n 8192 --m 32768 \\
        --fetch gpurun_out/pmc_FETCH_SIZE --write gpurun_out/pmc_WRITE_SIZE \\
        --copy-bytes 1073741824 --out profiles/mp_step_f32_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os


def _counter(path: str, kernel_substr: str) -> list:
    """The counter's value for each dispatch of the kernel, in dispatch order."""
    vals = []
    with open(path) as f:
        for row in csv.DictReader(f):
            if kernel_substr in row["Kernel_Name"]:
                vals.append((int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    if not vals:
        raise SystemExit(f"no dispatch of {kernel_substr} in {path}")
    return [v for _, v in sorted(vals)]


def _mean(vals) -> float:
    return sum(vals) / len(vals)


def pass_positions(fetch, min_fraction):
    """Dispatch positions kept when launches without a correlation pass are
    dropped: those whose FETCH_SIZE is at least min_fraction of the largest.
    (A decode that carries each step into the next launch ends with a launch
    that only applies the last step.)"""
    top = max(fetch)
    return [i for i, v in enumerate(fetch) if v >= min_fraction * top]


def source_sha(paths) -> str:
    """SHA-256 prefix over the kernel's source files, in the order given."""
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--source", required=True, action="append",
                    help="a source file the kernel is built from (repeat for each)")
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--m", type=int, required=True)
    ap.add_argument("--fetch", required=True, help="directory of the FETCH_SIZE runs")
    ap.add_argument("--write", required=True, help="directory of the WRITE_SIZE runs")
    ap.add_argument("--bench-prefix", default="bench")
    ap.add_argument("--copy-prefix", default="copy")
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--algorithmic-bytes", type=float, default=None)
    ap.add_argument("--pass-only", type=float, default=None, metavar="FRACTION",
                    help="drop dispatches whose FETCH_SIZE is below FRACTION of the largest "
                         "(launches that ran no correlation pass) from both runs")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    fv = _counter(os.path.join(a.fetch, f"{a.bench_prefix}_counter_collection.csv"), a.kernel)
    wv = _counter(os.path.join(a.write, f"{a.bench_prefix}_counter_collection.csv"), a.kernel)
    dropped = 0
    if a.pass_only is not None:
        if len(fv) != len(wv):
            raise SystemExit("FETCH and WRITE runs hold different dispatch counts")
        keep = pass_positions(fv, a.pass_only)
        dropped = len(fv) - len(keep)
        fv = [fv[i] for i in keep]
        wv = [wv[i] for i in keep]
    f_k, nf = _mean(fv), len(fv)
    w_k, nw = _mean(wv), len(wv)
    f_c = _mean(_counter(os.path.join(a.fetch, f"{a.copy_prefix}_counter_collection.csv"),
                         "k_copy"))
    w_c = _mean(_counter(os.path.join(a.write, f"{a.copy_prefix}_counter_collection.csv"),
                         "k_copy"))
    f_scale = a.copy_bytes / (f_c * 1024.0)
    w_scale = a.copy_bytes / (w_c * 1024.0)
    fetch = f_k * 1024.0 * f_scale
    write = w_k * 1024.0 * w_scale
    out = dict(kernel=a.kernel, kernel_sha=source_sha(a.source), n=a.n, m=a.m,
               fetch_kib_per_dispatch=f_k, write_kib_per_dispatch=w_k,
               dispatches=dict(fetch=nf, write=nw, dropped_without_pass=dropped),
               copy_fetch_kib=f_c, copy_write_kib=w_c, copy_bytes=a.copy_bytes,
               fetch_scale=f_scale, write_scale=w_scale,
               fetch_bytes_per_launch=round(fetch), write_bytes_per_launch=round(write),
               bytes_per_launch=round(fetch + write))
    if a.algorithmic_bytes:
        out["algorithmic_bytes_per_launch"] = a.algorithmic_bytes
        out["traffic_over_algorithmic"] = (fetch + write) / a.algorithmic_bytes
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
