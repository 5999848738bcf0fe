"""Mean of each counter per dispatch, per kernel, from a rocprofv3 --pmc run.

A counter run over thousands of dispatches writes one CSV row per counter
and dispatch; this reduces it to a few lines per kernel (and can delete the
raw file, which can be hundreds of MB).

    python -m paper_0809_1833_amd.probe.pmc_summary RUN_DIR --kernel k_bcorr \\
        --kernel k_bselect --out summary.json [--delete]
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os


def summarize(path: str, kernels) -> dict:
    sums = collections.defaultdict(lambda: collections.defaultdict(float))
    ids = collections.defaultdict(set)
    with open(path) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            if not any(k in name for k in kernels):
                continue
            key = name.split("(")[0]
            sums[key][row["Counter_Name"]] += float(row["Counter_Value"])
            ids[key].add(row["Dispatch_Id"])
    return {k: {"dispatches": len(ids[k]),
                "mean_per_dispatch": {c: v / len(ids[k]) for c, v in sorted(sums[k].items())}}
            for k in sums}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("run_dir")
    ap.add_argument("--kernel", action="append", required=True,
                    help="substring of the kernel names to keep (repeat for each)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--delete", action="store_true", help="remove the raw CSV afterwards")
    a = ap.parse_args()
    paths = glob.glob(os.path.join(a.run_dir, "**", "*counter_collection.csv"), recursive=True)
    if len(paths) != 1:
        raise SystemExit(f"expected one counter_collection.csv under {a.run_dir}, found {len(paths)}")
    out = summarize(paths[0], a.kernel)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
    if a.delete:
        os.remove(paths[0])


if __name__ == "__main__":
    main()
