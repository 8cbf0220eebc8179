#!/usr/bin/env python3
"""Rewrites the "a2_momentum" table of tests/golden/paper_constants.json from
the recursion of Algorithm A2 (section 2.1): t(-1) = t(0) = 1,
t(k+1) = (1 + sqrt(1 + 4 t(k)^2)) / 2, and the momentum coefficient of
iteration k, (t(k-1) - 1) / t(k), evaluated in double precision.  The other
entries of the file (the section 2.1 filters, the paper's timings) are
printed in the paper and typed from it; this script leaves them unchanged.

Run:  python tests/golden/make_paper_constants.py
"""
from __future__ import annotations

import json
import math
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_constants.json")
N = 6


def a2_table(n: int = N):
    """t(0..n-1) and the coefficients of iterations 0..n-1."""
    t_prev, t_cur = 1.0, 1.0
    ts, coef = [], []
    for _ in range(n):
        ts.append(t_cur)
        coef.append((t_prev - 1.0) / t_cur)
        t_prev, t_cur = t_cur, 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t_cur * t_cur))
    return ts, coef


def main() -> None:
    with open(PATH) as fh:
        gold = json.load(fh)
    ts, coef = a2_table()
    gold["a2_momentum"]["t"] = ts
    gold["a2_momentum"]["coefficient"] = coef
    gold["a2_momentum"]["_generated_by"] = "tests/golden/make_paper_constants.py"
    with open(PATH, "w") as fh:
        json.dump(gold, fh, indent=1)
        fh.write("\n")
    print("wrote", PATH)


if __name__ == "__main__":
    main()
