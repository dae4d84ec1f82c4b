"""Writes micro_exact.json: exact rational solutions of a hand-made micro SDA problem.

Calls only ``oracle.exact`` (exact Fraction arithmetic, no rounding).  The
problem: 8 samples, 6 binary features, a hand-written similarity graph, 4
labeled samples (2 per class); alpha in {0, 1/2, 1}; beta in {1/10, 1, 10}.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction as F

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle import exact  # noqa: E402

ROWS = [[0, 1, 3], [0, 2], [1, 2, 4], [0, 3, 5], [2, 4], [1, 5], [0, 1, 2, 3], [4, 5]]
EDGES = [(0, 3), (0, 6), (1, 4), (2, 4), (2, 6), (3, 6), (5, 7), (1, 2)]
LAB_IDX = [0, 2, 5, 6]
LAB_Y = [1, -1, -1, 1]
ALPHAS = ["0", "1/2", "1"]
BETAS = ["1/10", "1", "10"]


def main():
    out = {"n": 8, "d": 6, "rows": ROWS, "edges": EDGES, "lab_idx": LAB_IDX, "lab_y": LAB_Y, "cases": []}
    for a in ALPHAS:
        for b in BETAS:
            A, rhs = exact.system(8, 6, ROWS, EDGES, LAB_IDX, LAB_Y, F(a), F(b))
            w = exact.solve(A, rhs)
            out["cases"].append({"alpha": a, "beta": b,
                                 "b": [str(v) for v in rhs],
                                 "w": [str(v) for v in w],
                                 "w_float": [float(v) for v in w]})
    path = os.path.join(os.path.dirname(__file__), "micro_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
