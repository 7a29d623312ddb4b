"""Writes tests/golden/cube_h32_histories.json: the FP64 oracle's solves on
the unit cube (benchmark 4) at h = 1/32, p = 2 and 3, the sizes of the 3-D
workload, whose oracle setup is too slow to repeat inside a GPU test.

Calls only the oracle.  For each p: the relative residual history of the
stand-alone solve to 1e-8 from x0 = 0 and from the seeded uniform [-1, 1]
guess (numpy default_rng(0)), the iteration counts, and the final iterate at
32 evenly spaced unknowns plus its 2-norm.  Run from the repository root:
    python tests/golden/make_cube_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402


def main():
    o_def = O.Options()
    out = {"_source": "oracle/oracle.c via tests/golden/make_cube_golden.py (oracle defaults: ILUT(%g, %g), "
                      "rule 2 mode %d, nested dissection, nu1 = nu2 = 1, two h-multigrid cycles)"
                      % (o_def.tau, o_def.fill, o_def.limit_mode),
           "nel": 32, "tol": 1e-8, "cases": {}}
    for p in (2, 3):
        o = O.Oracle(3, p, 32)
        assert o.status == 0
        f = o.f()
        case = {"n": o.n, "f_norm": float(np.linalg.norm(f))}
        idx = np.linspace(0, o.n - 1, 32).astype(int)
        for kind in ("zero", "random"):
            x0 = np.zeros(o.n) if kind == "zero" else np.random.default_rng(0).uniform(-1, 1, o.n)
            x, st, it, hist = o.solve(f, x0=x0, tol=1e-8)
            case[kind] = {"status": int(st), "iterations": int(it), "hist": [float(h) for h in hist],
                          "x_norm": float(np.linalg.norm(x)), "x_idx": idx.tolist(),
                          "x_at": [float(x[i]) for i in idx]}
            print(p, kind, it, hist[-1], flush=True)
        out["cases"][str(p)] = case
    json.dump(out, open(os.path.join(ROOT, "tests", "golden", "cube_h32_histories.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
