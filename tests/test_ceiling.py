"""The adapted lane-occupancy ceiling (Section VII, Eq. 1) against values
computed by hand (CPU only).

The no-match closed form (reads with no common base, scores +1/-1/-1, reads
longer than X) fixes every width: anti-diagonal d computes d + 1 cells for
d = 1..X and 2X - d + 3 cells for d = X+1..2X+1, X^2 + 4X + 2 cells in all
over 2X + 1 anti-diagonals.  A one-register job issues 64 lanes on each, so
its ceiling is (X^2 + 4X + 2) / (64 (2X + 1)); at X = 100 the job starts in
the two-register tier (X + 4 > 56) and issues 128 lanes.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2002_05200_amd import ceiling as CE


def no_match_widths(x):
    return [d + 1 for d in range(1, x + 1)] + [2 * x - d + 3 for d in range(x + 1, 2 * x + 2)]


@pytest.mark.parametrize("x,lanes", [(1, 64), (2, 64), (10, 64), (50, 64), (100, 128)])
def test_no_match_closed_form(x, lanes):
    m = n = 3 * x + 5
    t0 = CE.initial_tier(m, n, x)
    assert CE.TIER_CELLS[t0] * 64 == lanes
    got = CE.ceiling([(no_match_widths(x), t0)])
    want = (x * x + 4 * x + 2) / (lanes * (2 * x + 1))
    assert got["cells"] == x * x + 4 * x + 2
    assert got["anti_diagonals"] == 2 * x + 1
    assert got["eq1_mean"] == pytest.approx(want, rel=1e-12)
    assert got["work_weighted"] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("x", [3, 10, 40])
def test_oracle_trace_feeds_the_closed_form(x):
    """The widths the oracle traces on a no-match pair are the hand-derived
    ones, so the ceiling computed from them is the closed form."""
    r = np.random.default_rng(x)
    m, n = 2 * x + 7, 3 * x + 4
    a = r.integers(0, 2, m).astype(np.uint8)         # A, C
    b = (r.integers(0, 2, n) + 2).astype(np.uint8)   # G, T
    tr = O.extend(a, b, 1, -1, -1, x=x, trace=True)["trace"]
    widths = (tr["hi"] - tr["lo"] + 1).tolist()
    assert widths == no_match_widths(x)
    got = CE.ceiling([(widths, CE.initial_tier(m, n, x))])
    assert got["eq1_mean"] == pytest.approx((x * x + 4 * x + 2) / (64 * (2 * x + 1)))


def test_escalation_prices_each_anti_diagonal_in_its_tier():
    # five ranges of 10 cells in the one-register tier, then ranges of 70
    # cells, which need the two-register window (62 slots at most before)
    widths = [10] * 5 + [70] * 3
    got = CE.ceiling([(widths, 0)])
    assert got["eq1_mean"] == pytest.approx((5 * 10 / 64 + 3 * 70 / 128) / 8)
    assert got["work_weighted"] == pytest.approx((50 + 210) / (5 * 64 + 3 * 128))
    t0 = CE.ceiling([(widths, 0)], only_tier=0)
    assert t0["anti_diagonals"] == 5 and t0["work_weighted"] == pytest.approx(10 / 64)


def test_wide_tiers_issue_only_the_spanned_registers():
    # 300 cells in the eight-register tier: ceil(300 / 64) + 1 = 6 registers
    got = CE.ceiling([([300, 300], 3)])
    assert got["lanes"] == 2 * 6 * 64
    # never more registers than the tier has
    assert CE.lanes_issued(np.array([500]), 4).tolist() == [256]
