"""Brute-force references that pin the C oracle (test helpers, CPU only).

``full_dp``: the plain full dynamic-programming matrix of the cell recurrence
(Section III-A) with no pruning at all; the best cell over the whole matrix.
With X at least the whole score range, X-drop never prunes and must equal it.

``xdrop_full``: X-drop written over an explicit full matrix, with -inf as
Python's ``-math.inf`` and each anti-diagonal's range found by scanning the
matrix.  It shares no code or data structure with the C oracle's rolling
anti-diagonals, so agreement pins the oracle's bookkeeping.

Both are pure-Python loops for tiny inputs.  Either takes match/mismatch
scores or, with ``table``, a 4 x 4 substitution table (table[x][y] scores
base x of a against base y of b).
"""
import math

NEG_INF = -math.inf


def score(x, y, match, mismatch, table=None):
    if table is not None:
        return table[x][y]
    return match if x == y else mismatch


def full_dp(a, b, match=1, mismatch=-1, gap=-1, table=None):
    m, n = len(a), len(b)
    S = [[0] * (n + 1) for _ in range(m + 1)]
    for i in range(m + 1):
        for j in range(n + 1):
            if i == 0 and j == 0:
                continue
            cands = []
            if i > 0 and j > 0:
                cands.append(S[i - 1][j - 1] + score(a[i - 1], b[j - 1], match, mismatch, table))
            if i > 0:
                cands.append(S[i - 1][j] + gap)
            if j > 0:
                cands.append(S[i][j - 1] + gap)
            S[i][j] = max(cands)
    # best cell: highest score; then earliest anti-diagonal; then smallest i
    best_key = None
    for i in range(m + 1):
        for j in range(n + 1):
            key = (-S[i][j], i + j, i)
            if best_key is None or key < best_key:
                best_key = key
    best, bi = -best_key[0], best_key[2]
    bj = best_key[1] - bi
    return {"best": best, "bi": bi, "bj": bj, "cells": (m + 1) * (n + 1) - 1, "S": S}


def xdrop_full(a, b, match=1, mismatch=-1, gap=-1, x=10, table=None):
    m, n = len(a), len(b)
    S = [[NEG_INF] * (n + 1) for _ in range(m + 1)]
    S[0][0] = 0
    best, bi, bj, cells = 0, 0, 0, 0
    ranges = []
    for d in range(1, m + n + 1):
        prev = [i for i in range(0, m + 1) if 0 <= d - 1 - i <= n and S[i][d - 1 - i] != NEG_INF]
        if not prev:
            break
        lo = max(min(prev), d - n)
        hi = min(max(prev) + 1, m)
        if lo > hi:
            break
        threshold = best - x
        for i in range(lo, hi + 1):
            j = d - i
            v = NEG_INF
            if i > 0 and j > 0:
                v = max(v, S[i - 1][j - 1] + score(a[i - 1], b[j - 1], match, mismatch, table))
            if i > 0:
                v = max(v, S[i - 1][j] + gap)
            if j > 0:
                v = max(v, S[i][j - 1] + gap)
            S[i][j] = v if v >= threshold else NEG_INF
        cells += hi - lo + 1
        ranges.append((d, lo, hi))
        row = [(S[i][d - i], i) for i in range(lo, hi + 1) if S[i][d - i] != NEG_INF]
        if row:
            top = max(v for v, _ in row)
            if top > best:
                best = top
                bi = min(i for v, i in row if v == top)
                bj = d - bi
    return {"best": int(best), "bi": bi, "bj": bj, "cells": cells, "S": S, "ranges": ranges}


def seed_pair(a, b, pa, pb, k, match=1, mismatch=-1, gap=-1, x=10, ext=xdrop_full):
    """Seed split of one pair with a brute-force extension."""
    r = ext(a[pa + k:], b[pb + k:], match, mismatch, gap, x)
    l = ext(a[:pa][::-1], b[:pb][::-1], match, mismatch, gap, x)
    seed = sum(score(a[pa + t], b[pb + t], match, mismatch) for t in range(k))
    return {"score": l["best"] + seed + r["best"], "left_score": l["best"],
            "right_score": r["best"], "seed_score": seed,
            "a_begin": pa - l["bi"], "a_end": pa + k + r["bi"],
            "b_begin": pb - l["bj"], "b_end": pb + k + r["bj"],
            "left_cells": l["cells"], "right_cells": r["cells"]}
