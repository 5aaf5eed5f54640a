"""Property tests of the oracles with hypothesis (CPU only).

Hypothesis draws the reads, scores and X and shrinks any failure to a
smallest case.  Each property is fixed by the mathematics of Section III-A or
by an independent brute force, never by the oracle itself:
  - X large enough that nothing is pruned: the full-matrix optimum with the
    end-cell tie-break (brute force, P1);
  - any X: the full-matrix X-drop written with explicit masks (P2);
  - swapping the reads swaps the end coordinates when the best cell is
    unique and keeps score and cells (P6);
  - scaling scores and X by c scales the score and keeps ends and cells (P7);
  - 0 <= best(X) <= best(no pruning), and X below -gap gives the origin (P9,
    P10);
  - the seed choice equals a brute force over all position pairs (S1).
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import brute
from oracle import oracle as O

SETTINGS = settings(max_examples=300, deadline=None,
                    suppress_health_check=[HealthCheck.too_slow])

reads = st.lists(st.integers(0, 3), min_size=0, max_size=14)
binary_reads = st.lists(st.integers(0, 1), min_size=0, max_size=12)
score_sets = st.tuples(st.integers(1, 4), st.integers(-4, 0), st.integers(-4, -1)).filter(
    lambda s: s[0] >= s[1])


def ext(a, b, sc, x):
    return O.extend(np.array(a, np.uint8), np.array(b, np.uint8), *sc, x=x)


@SETTINGS
@given(a=reads, b=reads, sc=score_sets)
def test_no_pruning_equals_full_dp(a, b, sc):
    got = ext(a, b, sc, 1 << 29)
    ref = brute.full_dp(a, b, *sc)
    assert (got["best"], got["bi"], got["bj"], got["cells"]) == \
        (ref["best"], ref["bi"], ref["bj"], ref["cells"])


@SETTINGS
@given(a=st.one_of(reads, binary_reads), b=st.one_of(reads, binary_reads), sc=score_sets,
       x=st.integers(0, 12))
def test_any_x_equals_full_matrix_xdrop(a, b, sc, x):
    got = ext(a, b, sc, x)
    ref = brute.xdrop_full(a, b, *sc, x=x)
    assert (got["best"], got["bi"], got["bj"], got["cells"]) == \
        (ref["best"], ref["bi"], ref["bj"], ref["cells"])


@SETTINGS
@given(a=reads, b=reads, sc=score_sets, x=st.integers(0, 12))
def test_swapping_the_reads(a, b, sc, x):
    ab, ba = ext(a, b, sc, x), ext(b, a, sc, x)
    assert ab["best"] == ba["best"] and ab["cells"] == ba["cells"]
    full = brute.xdrop_full(a, b, *sc, x=x)
    S = full["S"]
    d = ab["bi"] + ab["bj"]
    tops = [i for i in range(len(a) + 1) if 0 <= d - i <= len(b) and S[i][d - i] == ab["best"]]
    if len(tops) == 1:
        assert (ba["bi"], ba["bj"]) == (ab["bj"], ab["bi"])


@SETTINGS
@given(a=reads, b=reads, sc=score_sets, x=st.integers(0, 12), c=st.integers(2, 5))
def test_scaling_scores_and_x(a, b, sc, x, c):
    one = ext(a, b, sc, x)
    big = ext(a, b, tuple(c * s for s in sc), c * x)
    assert big["best"] == c * one["best"]
    assert (big["bi"], big["bj"], big["cells"]) == (one["bi"], one["bj"], one["cells"])


@SETTINGS
@given(a=reads, b=reads, sc=score_sets, x=st.integers(0, 12))
def test_sandwich_and_tiny_x(a, b, sc, x):
    got = ext(a, b, sc, x)
    top = brute.full_dp(a, b, *sc)["best"]
    assert 0 <= got["best"] <= top
    if x < -sc[2]:
        assert (got["best"], got["bi"], got["bj"]) == (0, 0, 0)
        assert got["cells"] == int(len(a) > 0) + int(len(b) > 0)


def brute_seed(a, b, k, width):
    matches = [(p, q) for p in range(len(a) - k + 1) for q in range(len(b) - k + 1)
               if a[p:p + k] == b[q:q + k]]
    if not matches:
        return (0, 0, 0, 0, 0)
    bins = {}
    for p, q in matches:
        bins.setdefault((q - p) // width, []).append((p, q))
    win = min(bins, key=lambda z: (-len(bins[z]), z))
    p, q = min(bins[win])
    return (p, q, len(bins[win]), len(matches), 1)


@SETTINGS
@given(a=st.lists(st.integers(0, 3), max_size=40), b=st.lists(st.integers(0, 3), max_size=40),
       k=st.integers(1, 6), width=st.integers(1, 15))
def test_seed_choice_equals_brute_force(a, b, k, width):
    got = O.find_seed(np.array(a, np.uint8), np.array(b, np.uint8), k=k, width=width)
    ref = brute_seed(a, b, k, width)
    assert (got["a_seed"], got["b_seed"], got["bin_matches"], got["matches"], got["found"]) == ref
    assert got["status"] == 0


@pytest.mark.parametrize("k,width", [(0, 5), (32, 5), (5, 0)])
def test_seed_choice_rejects_bad_arguments(k, width):
    got = O.find_seed(np.zeros(10, np.uint8), np.zeros(10, np.uint8), k=k, width=width)
    assert got["status"] == 1 and got["found"] == 0
