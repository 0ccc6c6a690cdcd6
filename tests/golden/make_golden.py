"""Writes tests/golden/draws.json from the reference checker only.

Each case stores a probability vector (as exact float hex strings), the draw
parameters and the sorted index set the checker's sampler returns.  Run from
the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.sampling import draw, probs_uniform, probs_length  # noqa: E402
import workloads  # noqa: E402


def main():
    cases = []
    p, q = probs_uniform(256, 256)
    cases.append(("uniform_256_c40_J", p, 40, 1, 0, False))
    cases.append(("uniform_256_r40_I", q, 40, 1, 1, False))
    A = workloads.color_like(96, 80, 6, seed=2)
    p, q, _ = probs_length(A)
    cases.append(("length_color_80_c24_J", p, 24, 2, 0, False))
    cases.append(("length_color_96_r24_I", q, 24, 2, 1, False))
    cases.append(("length_color_80_c30_repl", p, 30, 5, 0, True))
    rng = workloads.rng_for(99, 0)
    w = rng.random(1000) ** 4
    w /= w.sum()
    cases.append(("skewed_1000_c100", w, 100, 77, 3, False))
    out = []
    for name, pv, count, seed, set_id, repl in cases:
        idx = draw(pv, count, seed, set_id, repl)
        out.append(dict(name=name, p=[float(x).hex() for x in pv], count=count, seed=seed,
                        set_id=set_id, with_replacement=repl, idx=[int(i) for i in idx]))
    with open(os.path.join(ROOT, "tests", "golden", "draws.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", len(out), "cases")


if __name__ == "__main__":
    main()
