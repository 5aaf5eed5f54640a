"""Seeded synthetic read pairs for batched X-drop seed extension.

This module only draws inputs: random template reads, an error model
(substitutions, insertions, deletions), an exact k-mer seed shared by both
reads, and the X-drop threshold of each pair.  It holds none of the
extension arithmetic; the CPU oracle and the HIP library consume what it
returns and nothing else is shared between them.

The paper's own evaluation set (100K pairs of 2.5-7.5 kb reads with about 15%
error, Section VI-A) was never published; the workloads below are seeded
stand-ins with the shapes of the paper's workloads.

Every pair is generated from its own counter-addressed stream,
``SeedSequence(ROOT_SEED, spawn_key=(workload_id, pair_index))``, so any
subset of a workload can be regenerated independently and in parallel.

Bases are coded A=0, C=1, G=2, T=3 (uint8, one code per byte).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 200205200
SEED_K = 17
DEFAULT_SCORES = (1, -1, -1)  # match, mismatch, gap (linear)

_ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)


# ---------------------------------------------------------------------------
# batch container
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Batch:
    """A batch of read pairs laid out as two base arenas.

    ``a`` / ``b``: concatenated reads (uint8 codes 0..3).
    Pair ``p`` uses ``a[a_off[p] : a_off[p] + a_len[p]]`` and the analogous
    slice of ``b``; its seed is ``A[a_seed : a_seed + k] ~ B[b_seed : b_seed + k]``
    in read-local coordinates, and ``x[p]`` is its X-drop threshold.
    """

    a: np.ndarray
    b: np.ndarray
    a_off: np.ndarray
    a_len: np.ndarray
    b_off: np.ndarray
    b_len: np.ndarray
    a_seed: np.ndarray
    b_seed: np.ndarray
    x: np.ndarray
    k: int = SEED_K
    scores: Tuple[int, int, int] = DEFAULT_SCORES
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.a_len.shape[0])

    def pair(self, p: int) -> Tuple[np.ndarray, np.ndarray]:
        a = self.a[self.a_off[p]: self.a_off[p] + self.a_len[p]]
        b = self.b[self.b_off[p]: self.b_off[p] + self.b_len[p]]
        return a, b

    def subset(self, idx: Sequence[int]) -> "Batch":
        """A new, compact batch holding the pairs ``idx`` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        pairs = [self.pair(int(p)) for p in idx]
        return from_pairs(
            [p[0] for p in pairs], [p[1] for p in pairs],
            self.a_seed[idx], self.b_seed[idx], self.x[idx],
            k=self.k, scores=self.scores, name=self.name + "[subset]")

    def total_bases(self) -> int:
        return int(self.a_len.sum() + self.b_len.sum())


def from_pairs(a_list, b_list, a_seed, b_seed, x, k=SEED_K,
               scores=DEFAULT_SCORES, name="") -> Batch:
    """Lay out explicit read pairs as arenas."""
    a_len = np.array([len(s) for s in a_list], dtype=np.int64)
    b_len = np.array([len(s) for s in b_list], dtype=np.int64)
    a_off = np.zeros_like(a_len)
    b_off = np.zeros_like(b_len)
    if len(a_len):
        a_off[1:] = np.cumsum(a_len)[:-1]
        b_off[1:] = np.cumsum(b_len)[:-1]
    a = (np.concatenate([np.asarray(s, dtype=np.uint8) for s in a_list])
         if len(a_list) else np.zeros(0, np.uint8))
    b = (np.concatenate([np.asarray(s, dtype=np.uint8) for s in b_list])
         if len(b_list) else np.zeros(0, np.uint8))
    return Batch(a=a, b=b, a_off=a_off, a_len=a_len, b_off=b_off, b_len=b_len,
                 a_seed=np.asarray(a_seed, dtype=np.int64).reshape(-1),
                 b_seed=np.asarray(b_seed, dtype=np.int64).reshape(-1),
                 x=np.asarray(x, dtype=np.int32).reshape(-1),
                 k=int(k), scores=tuple(int(s) for s in scores), name=name)


def concat(batches: Sequence[Batch], name: str = "") -> Batch:
    """Concatenate batches that share k and scores."""
    assert batches
    k, sc = batches[0].k, batches[0].scores
    for bt in batches:
        assert bt.k == k and bt.scores == sc
    a_shift = np.cumsum([0] + [len(bt.a) for bt in batches[:-1]])
    b_shift = np.cumsum([0] + [len(bt.b) for bt in batches[:-1]])
    return Batch(
        a=np.concatenate([bt.a for bt in batches]),
        b=np.concatenate([bt.b for bt in batches]),
        a_off=np.concatenate([bt.a_off + s for bt, s in zip(batches, a_shift)]),
        a_len=np.concatenate([bt.a_len for bt in batches]),
        b_off=np.concatenate([bt.b_off + s for bt, s in zip(batches, b_shift)]),
        b_len=np.concatenate([bt.b_len for bt in batches]),
        a_seed=np.concatenate([bt.a_seed for bt in batches]),
        b_seed=np.concatenate([bt.b_seed for bt in batches]),
        x=np.concatenate([bt.x for bt in batches]),
        k=k, scores=sc, name=name or batches[0].name)


# ---------------------------------------------------------------------------
# random primitives
# ---------------------------------------------------------------------------
def pair_rng(workload_id: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(
        np.random.SeedSequence(ROOT_SEED, spawn_key=(int(workload_id),) + tuple(int(k) for k in key)))


def random_bases(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 4, size=int(n), dtype=np.uint8)


def mutate(rng: np.random.Generator, t: np.ndarray, p_sub: float, p_ins: float,
           p_del: float) -> np.ndarray:
    """Copy template ``t`` through a per-base error channel.

    For each template base one uniform draw u decides: u < p_del deletes it;
    u < p_del + p_sub replaces it by one of the other three bases (uniformly);
    u < p_del + p_sub + p_ins keeps it and inserts one uniform random base
    after it; otherwise it is kept.
    """
    n = len(t)
    u = rng.random(n)
    sub_shift = rng.integers(1, 4, size=n, dtype=np.uint8)
    ins_base = rng.integers(0, 4, size=n, dtype=np.uint8)
    if n == 0:
        return np.zeros(0, np.uint8)
    is_del = u < p_del
    is_sub = (~is_del) & (u < p_del + p_sub)
    is_ins = (~is_del) & (~is_sub) & (u < p_del + p_sub + p_ins)
    kept = np.where(is_sub, (t + sub_shift) & 3, t).astype(np.uint8)
    counts = np.where(is_del, 0, np.where(is_ins, 2, 1))
    start = np.cumsum(counts) - counts
    out = np.empty(int(counts.sum()), dtype=np.uint8)
    live = ~is_del
    out[start[live]] = kept[live]
    out[start[is_ins] + 1] = ins_base[is_ins]
    return out


def log_uniform_len(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def true_pair(rng, length: int, seed_pos: Optional[int], p_sub, p_ins, p_del,
              k: int = SEED_K):
    """Read A and a noisy copy B that share A's k-mer at ``seed_pos`` exactly."""
    a = random_bases(rng, length)
    if seed_pos is None:
        seed_pos = int(rng.integers(0, length - k + 1))
    left = mutate(rng, a[:seed_pos], p_sub, p_ins, p_del)
    right = mutate(rng, a[seed_pos + k:], p_sub, p_ins, p_del)
    b = np.concatenate([left, a[seed_pos:seed_pos + k], right])
    return a, b, seed_pos, len(left)


def spurious_pair(rng, len_a: int, len_b: int, k: int = SEED_K):
    """Independent random reads that share only one planted k-mer."""
    a = random_bases(rng, len_a)
    b = random_bases(rng, len_b)
    pa = int(rng.integers(0, len_a - k + 1))
    pb = int(rng.integers(0, len_b - k + 1))
    b[pb:pb + k] = a[pa:pa + k]
    return a, b, pa, pb


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    wid: int
    name: str
    n_pairs: int
    x: int
    describe: str


WORKLOADS: Dict[str, Workload] = {
    "plain1k": Workload(1, "plain1k", 1000, 10,
                        "1,000 pairs, |A|=1,000, B = A with 5% sub / 5% ins / 5% del, "
                        "exact 17-mer seed at A[450..533], X=10"),
    "batch10k": Workload(2, "batch10k", 100000, 50,
                         "100,000 pairs, |A| log-normal (median 10 kb, sigma_ln 0.5) "
                         "clipped to [1 kb, 40 kb], 15% error split evenly, X=50"),
    "uneven": Workload(3, "uneven", 200000, 100,
                       "200,000 pairs, |A| log-uniform 0.5-100 kb; half true overlaps "
                       "(10-15% error split evenly), half spurious (independent B sharing "
                       "only the 17-mer seed), X=100"),
    "serving": Workload(4, "serving", 0, 0,
                        "Poisson requests of 1-64 pairs, log-uniform 0.5-50 kb, 12% error "
                        "split evenly, X per request from {10, 50, 100}"),
    "ultralong": Workload(5, "ultralong", 2000, 1000,
                          "2,000 pairs, |A| log-uniform 100 kb-1 Mb, 5% error split evenly, "
                          "X=1000"),
}


def make_pair(workload: str, idx: int):
    """Pair ``idx`` of a batch workload: (A, B, a_seed, b_seed, X)."""
    w = WORKLOADS[workload]
    rng = pair_rng(w.wid, idx)
    if workload == "plain1k":
        pa = int(rng.integers(450, 534))
        a, b, pa, pb = true_pair(rng, 1000, pa, 0.05, 0.05, 0.05)
        return a, b, pa, pb, w.x
    if workload == "batch10k":
        length = int(round(rng.lognormal(math.log(10000.0), 0.5)))
        length = min(max(length, 1000), 40000)
        a, b, pa, pb = true_pair(rng, length, None, 0.05, 0.05, 0.05)
        return a, b, pa, pb, w.x
    if workload == "uneven":
        spurious = bool(rng.random() < 0.5)
        la = log_uniform_len(rng, 500, 100000)
        if spurious:
            lb = log_uniform_len(rng, 500, 100000)
            a, b, pa, pb = spurious_pair(rng, la, lb)
        else:
            e = rng.uniform(0.10, 0.15) / 3.0
            a, b, pa, pb = true_pair(rng, la, None, e, e, e)
        return a, b, pa, pb, w.x
    if workload == "ultralong":
        la = log_uniform_len(rng, 100000, 1000000)
        e = 0.05 / 3.0
        a, b, pa, pb = true_pair(rng, la, None, e, e, e)
        return a, b, pa, pb, w.x
    raise KeyError(f"{workload} is not a batch workload")


def _chunk(args):
    workload, lo, hi = args
    ps = [make_pair(workload, i) for i in range(lo, hi)]
    return from_pairs([p[0] for p in ps], [p[1] for p in ps], [p[2] for p in ps],
                      [p[3] for p in ps], [p[4] for p in ps], name=workload)


def make_batch(workload: str, n: Optional[int] = None, start: int = 0,
               workers: int = 1, stride: int = 1) -> Batch:
    """Pairs ``start, start+stride, ...`` (``n`` of them) of a batch workload.

    ``stride > 1`` draws an evenly spread sample of the workload (used for the
    bounded CPU-baseline sample).  ``workers > 1`` generates in a process pool
    (fork); pair contents do not depend on ``workers``.
    """
    w = WORKLOADS[workload]
    if n is None:
        n = w.n_pairs
    if stride != 1:
        idx = [start + i * stride for i in range(n)]
        ps = [make_pair(workload, i) for i in idx]
        return from_pairs([p[0] for p in ps], [p[1] for p in ps], [p[2] for p in ps],
                          [p[3] for p in ps], [p[4] for p in ps], name=workload)
    if workers <= 1 or n < 256:
        return _chunk((workload, start, start + n))
    step = max(64, (n + workers * 8 - 1) // (workers * 8))
    jobs = [(workload, s, min(s + step, start + n)) for s in range(start, start + n, step)]
    return concat(pool_map(_chunk, jobs, workers), name=workload)


def pool_map(fn, jobs, workers: int, chunksize: int = 1) -> list:
    """``fn`` over ``jobs`` in a pool of ``workers`` forked processes.  The
    pool is closed and joined, so the workers leave on their own: a pool
    left by ``with`` terminates them with SIGTERM, which a profiler's signal
    handler preloaded into every process (rocprofv3) may not return from."""
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(workers)
    try:
        out = pool.map(fn, jobs, chunksize=chunksize)
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return out


# ---------------------------------------------------------------------------
# serving workload: requests and arrivals
# ---------------------------------------------------------------------------
SERVING_X = (10, 50, 100)


def make_request(req: int) -> Batch:
    """Request ``req`` of the serving workload: 1-64 pairs sharing one X."""
    w = WORKLOADS["serving"]
    hdr = pair_rng(w.wid, 0, req)
    n_pairs = int(hdr.integers(1, 65))
    x = SERVING_X[int(hdr.integers(0, len(SERVING_X)))]
    a_l, b_l, pa_l, pb_l = [], [], [], []
    for p in range(n_pairs):
        rng = pair_rng(w.wid, 1, req, p)
        la = log_uniform_len(rng, 500, 50000)
        a, b, pa, pb = true_pair(rng, la, None, 0.04, 0.04, 0.04)
        a_l.append(a); b_l.append(b); pa_l.append(pa); pb_l.append(pb)
    return from_pairs(a_l, b_l, pa_l, pb_l, [x] * n_pairs, name=f"serving[{req}]")


def poisson_arrivals(n: int, rate_per_s: float, seed_key: int = 0) -> np.ndarray:
    """Arrival times (seconds from start) of ``n`` requests at ``rate_per_s``."""
    rng = pair_rng(WORKLOADS["serving"].wid, 2, seed_key)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    return np.cumsum(gaps)


# ---------------------------------------------------------------------------
# small random cases for tests
# ---------------------------------------------------------------------------
def random_cases(seed: int, n: int, len_lo: int, len_hi: int, err: float = 0.15,
                 x_choices=(0, 1, 2, 5, 10, 20, 50), k: int = SEED_K,
                 spurious_frac: float = 0.25, scores=DEFAULT_SCORES) -> Batch:
    """Mixed small pairs: true overlaps, spurious pairs, edge seeds, short reads."""
    rng = np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=(99, seed)))
    a_l, b_l, pa_l, pb_l, x_l = [], [], [], [], []
    for _ in range(n):
        la = int(rng.integers(max(len_lo, k), max(len_hi, k) + 1))
        kind = rng.random()
        if kind < spurious_frac:
            lb = int(rng.integers(max(len_lo, k), max(len_hi, k) + 1))
            a, b, pa, pb = spurious_pair(rng, la, lb, k)
        else:
            where = rng.random()
            if where < 0.1:
                pos = 0                      # seed at the start: empty left job
            elif where < 0.2:
                pos = la - k                 # seed at the end: empty right job
            else:
                pos = None
            e = float(rng.uniform(0.0, err)) / 3.0
            a, b, pa, pb = true_pair(rng, la, pos, e, e, e, k)
        a_l.append(a); b_l.append(b); pa_l.append(pa); pb_l.append(pb)
        x_l.append(int(x_choices[int(rng.integers(0, len(x_choices)))]))
    return from_pairs(a_l, b_l, pa_l, pb_l, x_l, k=k, scores=scores, name=f"random[{seed}]")


def decode(codes: np.ndarray) -> bytes:
    return _ALPHABET[np.asarray(codes, dtype=np.uint8)].tobytes()


def encode(text: str) -> np.ndarray:
    lut = np.full(256, 255, dtype=np.uint8)
    for i, ch in enumerate(b"ACGT"):
        lut[ch] = i
    out = lut[np.frombuffer(text.encode(), dtype=np.uint8)]
    if (out == 255).any():
        raise ValueError("non-ACGT character")
    return out
