"""Compile the C oracle into ``oracle/libmporacle.so`` with gcc.

Test infrastructure: the library built here is loaded only by the tests, the
smoke check and the benchmark's CPU-baseline leg.

The flags keep the build portable to any x86-64 host (no -march=native: the
shared object may run on a different machine than the one that built it) and
forbid FMA contraction, so every inner product is the plain sequential FP64
sum the source spells out.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mp_oracle.c")
OUT = os.path.join(HERE, "libmporacle.so")

CFLAGS = ["-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]


def build(verbose: bool = False, src: str = SRC, out: str = OUT) -> str:
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
