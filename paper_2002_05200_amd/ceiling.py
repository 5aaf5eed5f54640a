"""Adapted lane-occupancy ceiling of the X-drop kernels (Section VII, Eq. 1).

The paper prices its kernel not against the raw INT32 peak but against a
ceiling adapted to X-drop: the peak scaled by the share of the issued thread
slots that hold cells, averaged over the parallel iterations (anti-diagonals).
Printed, Eq. 1 divides the operations of each iteration by the number of
issue rounds its threads need; the reading taken here is the per-iteration
useful fraction

    ceiling = peak * (1/N) * sum_i  W_i / T_i

where W_i is the number of cells computed on anti-diagonal i (the width of
its computed range) and T_i the lanes the kernel issues for it.  Alongside,
the work-weighted form sum_i W_i / sum_i T_i is reported, which is what bounds
a throughput measured in cells per second.

Lanes issued per anti-diagonal, by the tier a job runs in (window of 64 * C
diagonal slots on one wavefront, C = 1, 2, 4, ..., 32):
  * C = 1: all 64 lanes of the single register, every anti-diagonal;
  * C = 2: both registers (128 lanes), every anti-diagonal;
  * C >= 4: only the registers the computed range spans; modelled as
    min(C, ceil(W / 64) + 1) registers (a range of W slots usually straddles
    one more register boundary than W / 64).
A job starts in the tier its X and read lengths select and moves to the next
one when its range needs more than 64 * C - 2 slots; it continues there (the
state is saved), so each anti-diagonal is priced in the tier that computed it.

Widths come from any trace of the computed ranges; the benchmark takes them
from the CPU oracle's per-anti-diagonal trace.  This module only does the
counting; it imports neither the oracle nor the HIP library.
"""
from __future__ import annotations

from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

WAVE = 64
TIER_CELLS = (1, 2, 4, 8, 16, 32)


def initial_tier(m: int, n: int, x: int) -> int:
    """The first tier of a job of an m x n matrix at threshold X: the band
    never exceeds min(m, n) + 1 cells and is typically about X + 4 wide."""
    w = min(min(m, n) + 1, x + 4)
    t = 0
    while t < len(TIER_CELLS) - 1 and w > WAVE * TIER_CELLS[t] - 8:
        t += 1
    return t


def lanes_issued(width: np.ndarray, c: int) -> np.ndarray:
    """Lanes one wavefront of C registers issues for ranges of these widths."""
    if c <= 2:
        return np.full(width.shape, WAVE * c, dtype=np.int64)
    regs = np.minimum(c, -(-width // WAVE) + 1)
    return WAVE * regs.astype(np.int64)


def job_lanes(widths: Sequence[int], tier0: int) -> Tuple[np.ndarray, np.ndarray]:
    """Per-anti-diagonal (cells, lanes) of one job that starts at tier0 and
    escalates when a range outgrows its window."""
    w = np.asarray(widths, dtype=np.int64)
    lanes = np.zeros_like(w)
    t = tier0
    start = 0
    while start < len(w):
        if t >= len(TIER_CELLS):          # wider than one wavefront: not priced here
            lanes[start:] = 0
            break
        cap = WAVE * TIER_CELLS[t] - 2
        over = np.nonzero(w[start:] > cap)[0]
        stop = start + int(over[0]) if len(over) else len(w)
        lanes[start:stop] = lanes_issued(w[start:stop], TIER_CELLS[t])
        start = stop
        t += 1
    return w, lanes


def ceiling(jobs: Iterable[Tuple[Sequence[int], int]], only_tier: Optional[int] = None) -> dict:
    """Adapted ceiling (fraction of the peak) over jobs given as
    (widths of their computed anti-diagonals, initial tier).  With only_tier,
    only the anti-diagonals computed in that tier count."""
    ratio_sum = 0.0
    n_iter = 0
    cells = 0
    lanes = 0
    for widths, t0 in jobs:
        if len(widths) == 0:
            continue
        w, l = job_lanes(widths, t0)
        if only_tier is not None:
            keep = np.zeros(len(w), dtype=bool)
            t = t0
            start = 0
            while start < len(w) and t < len(TIER_CELLS):
                cap = WAVE * TIER_CELLS[t] - 2
                over = np.nonzero(w[start:] > cap)[0]
                stop = start + int(over[0]) if len(over) else len(w)
                if t == only_tier:
                    keep[start:stop] = True
                start = stop
                t += 1
            w, l = w[keep], l[keep]
        ok = l > 0
        ratio_sum += float((w[ok] / l[ok]).sum())
        n_iter += int(ok.sum())
        cells += int(w[ok].sum())
        lanes += int(l[ok].sum())
    return {"eq1_mean": ratio_sum / n_iter if n_iter else 0.0,
            "work_weighted": cells / lanes if lanes else 0.0,
            "anti_diagonals": n_iter, "cells": cells, "lanes": lanes}
