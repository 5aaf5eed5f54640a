"""Pins of the oracle's substitution-table form (CPU only).

The cell recurrence of Section III-A with the match/mismatch choice replaced
by a 4 x 4 table (the generalisation Section VIII names as future work).  Each
test names what it pins:
  M1  brute force: with X beyond the score range, the full-DP best cell under
      the same table (recurrence with a table, table orientation, tie-break).
  M2  the independent full-matrix X-drop under the table, random tiny inputs
      and X (pruning, trimming, range rule with a table).
  M3  scaling table, gap and X by c scales the score and keeps ends and cells.
  M4  swapping the reads and transposing the table keeps score and cells.
  M5  identical reads under a table with a positive diagonal, non-positive
      off-diagonal entries and X >= -gap: best = sum of the diagonal entries
      of the read's bases, at (L, L) (the diagonal path rises on every even
      anti-diagonal and every odd one keeps a survivor).
  M6  the match/mismatch form is the table with match on its diagonal.
"""
import numpy as np
import pytest

import brute
from oracle import oracle as O

X_INF = 1 << 29


def rand_table(r, lo=-4, hi=5):
    return r.integers(lo, hi, (4, 4)).astype(np.int64)


def key(d):
    return (d["best"], d["bi"], d["bj"], d["cells"])


def test_m1_xinf_equals_full_dp():
    r = np.random.default_rng(21)
    for _ in range(200):
        t = rand_table(r)
        gap = -int(r.integers(1, 4))
        m, n = int(r.integers(0, 10)), int(r.integers(0, 10))
        a, b = list(r.integers(0, 4, m)), list(r.integers(0, 4, n))
        got = O.extend_matrix(np.array(a, np.uint8), np.array(b, np.uint8), t, gap, X_INF)
        ref = brute.full_dp(a, b, gap=gap, table=t.tolist())
        assert key(got) == key(ref), (a, b, t.tolist(), gap)


def test_m2_full_matrix_xdrop_random():
    r = np.random.default_rng(22)
    for _ in range(300):
        t = rand_table(r)
        gap = -int(r.integers(0, 4))
        m, n = int(r.integers(0, 25)), int(r.integers(0, 25))
        a = list(r.integers(0, 4, m))
        if r.random() < 0.6 and m:
            b = [c if r.random() > 0.2 else int(r.integers(0, 4)) for c in a][:n]
        else:
            b = list(r.integers(0, 4, n))
        x = int(r.integers(0, 15))
        got = O.extend_matrix(np.array(a, np.uint8), np.array(b, np.uint8), t, gap, x)
        ref = brute.xdrop_full(a, b, gap=gap, x=x, table=t.tolist())
        assert key(got) == key(ref), (a, b, t.tolist(), gap, x)


@pytest.mark.parametrize("c", [2, 3, 7])
def test_m3_scale_invariance(c):
    r = np.random.default_rng(23 + c)
    for _ in range(60):
        t = rand_table(r)
        gap = -int(r.integers(1, 4))
        a = r.integers(0, 4, int(r.integers(5, 200))).astype(np.uint8)
        b = a.copy() if r.random() < 0.5 else r.integers(0, 4, int(r.integers(5, 200))).astype(np.uint8)
        x = int(r.integers(0, 30))
        one = O.extend_matrix(a, b, t, gap, x)
        sc = O.extend_matrix(a, b, c * t, c * gap, c * x)
        assert sc["best"] == c * one["best"]
        assert (sc["bi"], sc["bj"], sc["cells"]) == (one["bi"], one["bj"], one["cells"])


def test_m4_swap_with_transposed_table():
    r = np.random.default_rng(24)
    for _ in range(100):
        t = rand_table(r)
        gap = -int(r.integers(1, 4))
        a = r.integers(0, 4, int(r.integers(1, 150))).astype(np.uint8)
        b = r.integers(0, 4, int(r.integers(1, 150))).astype(np.uint8)
        x = int(r.integers(0, 25))
        p = O.extend_matrix(a, b, t, gap, x)
        q = O.extend_matrix(b, a, t.T, gap, x)
        assert (p["best"], p["cells"]) == (q["best"], q["cells"])


def test_m5_identical_reads_closed_form():
    r = np.random.default_rng(25)
    for _ in range(40):
        t = -r.integers(0, 5, (4, 4)).astype(np.int64)
        np.fill_diagonal(t, r.integers(1, 9, 4))
        gap = -int(r.integers(1, 5))
        L = int(r.integers(0, 400))
        a = r.integers(0, 4, L).astype(np.uint8)
        for x in (-gap, -gap + 3, 100):
            got = O.extend_matrix(a, a, t, gap, x)
            assert got["best"] == int(t[a, a].sum())
            assert (got["bi"], got["bj"]) == (L, L)
        if L <= 12:
            ref = brute.full_dp(list(a), list(a), gap=gap, table=t.tolist())
            assert ref["best"] == int(t[a, a].sum())


def test_m6_linear_scores_are_the_diagonal_table():
    r = np.random.default_rng(26)
    for _ in range(60):
        match, mismatch, gap = int(r.integers(1, 6)), -int(r.integers(0, 6)), -int(r.integers(1, 4))
        t = np.full((4, 4), mismatch, np.int64)
        np.fill_diagonal(t, match)
        a = r.integers(0, 4, int(r.integers(0, 300))).astype(np.uint8)
        b = r.integers(0, 4, int(r.integers(0, 300))).astype(np.uint8)
        x = int(r.integers(0, 40))
        lin = O.extend(a, b, match, mismatch, gap, x)
        tab = O.extend_matrix(a, b, t, gap, x)
        assert key(lin) == key(tab)
        # and by brute force on a prefix small enough for it
        ref = brute.xdrop_full(list(a[:9]), list(b[:9]), match, mismatch, gap, x)
        assert key(O.extend(a[:9], b[:9], match, mismatch, gap, x)) == key(ref)
