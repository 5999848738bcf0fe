"""Write the stored expected values under tests/golden/.

Every expected value here comes from the exact rational MP in
``oracle/exact.py`` (Section 3, eqs. 8-12 with the smallest-index argmax of
eq. 16), run on seeded inputs from ``mpgen``.  Nothing is taken from the GPU
library.  Re-run with ``python tests/golden/make_golden.py`` to regenerate.
"""
from __future__ import annotations

import json
import os
import sys
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mpgen  # noqa: E402
from oracle.exact import exact_mp  # noqa: E402

# Small dictionaries with exactly unit-norm rational columns; y is an
# integer combination of three atoms so that the exact residual is rational.
CASES = [
    dict(name="stereo_n6_m10_s0", seed=0, n=6, m=10, atoms=(2, 5, 7), coefs=(3, -2, 1), iters=8),
    dict(name="stereo_n5_m12_s1", seed=1, n=5, m=12, atoms=(0, 4, 11), coefs=(1, 1, -4), iters=8),
    dict(name="stereo_n8_m16_s2", seed=2, n=8, m=16, atoms=(3, 9, 10), coefs=(-5, 2, 2), iters=7),
]


def rational_case(seed, n, m, atoms, coefs):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([900, seed])))
    cols = mpgen.rational_unit_dictionary(rng, n, m)
    y = [sum(Fraction(c) * cols[a][i] for a, c in zip(atoms, coefs)) for i in range(n)]
    return cols, y


def main():
    out = []
    for case in CASES:
        cols, y = rational_case(case["seed"], case["n"], case["m"], case["atoms"], case["coefs"])
        res = exact_mp(cols, y, Fraction(0), case["iters"])
        out.append(dict(
            case,
            idx=res["idx"],
            coef=[str(v) for v in res["coef"]],
            rr=[str(v) for v in res["rr"]],
            gap=[str(v) for v in res["gap"]],
            iters=res["iters"],
            reason=res["reason"],
        ))
    path = os.path.join(HERE, "exact_mp_stereographic.json")
    with open(path, "w") as f:
        json.dump(dict(
            source="exact rational Matching Pursuit (Section 3, eqs. 8-12; "
                   "argmax ties to the smallest index, eq. 16) on mpgen.rational_unit_dictionary "
                   "inputs seeded with SeedSequence([900, seed]); eps = 0, so each run stops at "
                   "its iteration cap",
            cases=out), f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
