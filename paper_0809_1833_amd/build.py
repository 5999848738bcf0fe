"""Build libmp.so (the HIP decoder and its C ABI) for gfx950 with hipcc.

``python -m paper_0809_1833_amd.build`` compiles every ``csrc/*.hip`` file
and links them into ``paper_0809_1833_amd/libmp.so`` next to this file.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmp.so")
PROBE_SRC = os.path.join(HERE, "probe", "stream_probe.hip")
PROBE = os.path.join(HERE, "probe", "stream_probe")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile all sources (in parallel) and link libmp.so; returns its path."""
    objdir = tempfile.mkdtemp(prefix="mpbuild_")
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    errors = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature; that note is expected
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            errors.append(f"{src}:\n{out}")
        elif out.strip() and verbose:
            print(out)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-shared", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(objdir)
    build_probe(verbose)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """The streaming-bandwidth / counter-calibration probe (an executable)."""
    tmp = PROBE + ".tmp"
    cmd = [HIPCC, *FLAGS, PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("probe build failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
