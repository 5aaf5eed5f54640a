"""Writes the stored fixtures of tests/golden.  Calls only the oracle.

no_match_cells.json -- closed form derived by hand (not computed by any code):
  reads with no common base, scores +1/-1/-1, m, n >= X + 1.  A cell (i, j)
  then scores -max(i, j) (Section III-A recurrence), so it survives iff
  max(i, j) <= X while best stays 0.  Anti-diagonals 1..X are computed whole
  (d + 1 cells each); anti-diagonal d in X+1..2X+1 gets the range
  [d-1-X, X+1] (2X - d + 3 cells) and 2X + 1 is the last.  Total
  X(X+1)/2 + X + (X+2)(X+3)/2 - 1 = X^2 + 4X + 2.

x_non_monotone.json -- a smallest-found pair of tiny reads where a smaller X
  gives a higher final score than a larger X, found by a seeded search with
  the oracle.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import oracle as O  # noqa: E402


def no_match():
    rows = [{"X": x, "cells": x * x + 4 * x + 2, "anti_diagonals": 2 * x + 1}
            for x in (1, 2, 3, 5, 10, 20, 50)]
    return {"source": "closed form derived by hand from the cell recurrence and the "
                      "X-drop rule (Section III-A); see make_golden.py",
            "scores": [1, -1, -1], "rows": rows}


def non_monotone():
    """Reads B made of (slightly edited) blocks copied from A, so that detours
    along other diagonals exist; the smallest hit of a seeded search is kept."""
    r = np.random.default_rng(2)
    score_sets = [(1, -1, -1), (1, -2, -1), (2, -1, -1), (1, -3, -2), (3, -2, -1)]
    best = None
    for _ in range(150000):
        m = int(r.integers(6, 30))
        a = r.integers(0, 4, m)
        segs = []
        for _ in range(int(r.integers(1, 4))):
            s = int(r.integers(0, m))
            L = int(r.integers(1, m - s + 1))
            seg = a[s:s + L].copy()
            if r.random() < 0.5:
                p = int(r.integers(0, L))
                seg[p] = (seg[p] + 1) % 4
            segs.append(seg)
            if r.random() < 0.5:
                segs.append(r.integers(0, 4, int(r.integers(0, 3))))
        b = np.concatenate(segs)
        xs = int(r.integers(0, 8))
        xl = xs + int(r.integers(1, 8))
        sc = score_sets[int(r.integers(0, len(score_sets)))]
        lo = O.extend(a, b, *sc, x=xs)["best"]
        hi = O.extend(a, b, *sc, x=xl)["best"]
        if lo > hi:
            key = (len(a) + len(b), xs, xl)
            if best is None or key < best[0]:
                best = (key, a.tolist(), b.tolist(), xs, xl, lo, hi, sc)
    assert best is not None
    _, a, b, xs, xl, lo, hi, sc = best
    return {"source": "seeded search over tiny reads with the oracle (make_golden.py)",
            "scores": list(sc), "a": a, "b": b, "x_small": xs, "x_large": xl,
            "best_small": lo, "best_large": hi}


if __name__ == "__main__":
    with open(os.path.join(HERE, "no_match_cells.json"), "w") as f:
        json.dump(no_match(), f, indent=1)
    with open(os.path.join(HERE, "x_non_monotone.json"), "w") as f:
        json.dump(non_monotone(), f, indent=1)
