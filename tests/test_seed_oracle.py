"""Pins of the seed-choice oracle (CPU only).

The reading of the binning seed choice (Section V): every exact k-mer match
(p, q) lies on diagonal q - p; diagonals are binned in bands of `width`; the
bin with the most matches wins (ties: the lower bin) and its match with the
smallest p, then q, is the seed.
  S1  brute force: all position pairs compared directly on tiny reads over
      two letters (many matches, many ties), every k and width small.
  S2  identical random reads: every match on diagonal 0, the seed is (0, 0)
      and there are |A| - k + 1 matches.
  S3  unrelated random reads sharing one planted k-mer: the first k-mer of
      the exact run holding it is the seed, and that run's k-mers are the
      only matches.
  S4  reads sharing no k-mer (disjoint alphabets) or shorter than k: no seed.
  S5  two planted runs on different diagonals: the longer run's bin wins.
"""
import numpy as np
import pytest

from oracle import oracle as O


def brute_seed(a, b, k, width):
    a, b = list(a), list(b)
    matches = [(p, q) for p in range(len(a) - k + 1) for q in range(len(b) - k + 1)
               if a[p:p + k] == b[q:q + k]]
    if not matches:
        return None
    bins = {}
    for p, q in matches:
        bins.setdefault((q - p) // width, []).append((p, q))   # // is floor division
    win = min(bins, key=lambda z: (-len(bins[z]), z))
    p, q = min(bins[win])
    return {"a_seed": p, "b_seed": q, "bin_matches": len(bins[win]), "matches": len(matches)}


def test_s1_brute_force_tiny():
    r = np.random.default_rng(41)
    for _ in range(1500):
        k = int(r.integers(1, 7))
        width = int(r.integers(1, 12))
        a = r.integers(0, 2, int(r.integers(0, 40)))
        b = r.integers(0, 2, int(r.integers(0, 40)))
        if r.random() < 0.3:
            b = np.concatenate([r.integers(0, 2, int(r.integers(0, 8))), a])[: len(b) + 5]
        got = O.find_seed(a, b, k=k, width=width)
        ref = brute_seed(a, b, k, width)
        if ref is None:
            assert got["found"] == 0 and got["matches"] == 0
        else:
            assert got["found"] == 1
            assert {f: got[f] for f in ref} == ref, (a.tolist(), b.tolist(), k, width)


def test_s2_identical_reads():
    r = np.random.default_rng(42)
    for L in (17, 18, 100, 1000, 3000):
        a = r.integers(0, 4, L).astype(np.uint8)
        got = O.find_seed(a, a, k=17, width=500)
        assert (got["found"], got["a_seed"], got["b_seed"]) == (1, 0, 0)
        assert got["matches"] == got["bin_matches"] == L - 17 + 1


def test_s3_planted_kmer():
    r = np.random.default_rng(43)
    for _ in range(20):
        a = r.integers(0, 4, int(r.integers(100, 2000))).astype(np.uint8)
        b = r.integers(0, 4, int(r.integers(100, 2000))).astype(np.uint8)
        p = int(r.integers(0, len(a) - 16))
        q = int(r.integers(0, len(b) - 16))
        b[q:q + 17] = a[p:p + 17]
        # the planted k-mer may extend by chance into a longer exact run on
        # its diagonal; the run's first k-mer is the seed
        p0, q0 = p, q
        while p0 > 0 and q0 > 0 and a[p0 - 1] == b[q0 - 1]:
            p0, q0 = p0 - 1, q0 - 1
        p1, q1 = p + 17, q + 17
        while p1 < len(a) and q1 < len(b) and a[p1] == b[q1]:
            p1, q1 = p1 + 1, q1 + 1
        got = O.find_seed(a, b, k=17, width=500)
        assert (got["found"], got["a_seed"], got["b_seed"]) == (1, p0, q0)
        assert got["matches"] == got["bin_matches"] == p1 - p0 - 17 + 1


def test_s4_no_seed():
    r = np.random.default_rng(44)
    a = r.integers(0, 2, 500).astype(np.uint8)          # A and C only
    b = (r.integers(0, 2, 500) + 2).astype(np.uint8)    # G and T only
    assert O.find_seed(a, b)["found"] == 0
    assert O.find_seed(a[:16], a[:16], k=17)["found"] == 0
    assert O.find_seed(a, a, k=0)["status"] == 1


def test_s5_the_longer_run_wins():
    r = np.random.default_rng(45)
    a = r.integers(0, 4, 3000).astype(np.uint8)
    b = r.integers(0, 4, 3000).astype(np.uint8)
    b[2000:2030] = a[100:130]      # 14 matches on diagonal 1900
    b[50:110] = a[1500:1560]       # 44 matches on diagonal -1450
    got = O.find_seed(a, b, k=17, width=100)
    assert (got["a_seed"], got["b_seed"], got["bin_matches"]) == (1500, 50, 44)
