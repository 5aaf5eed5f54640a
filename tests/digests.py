"""Chunk digests of whole workloads (test helpers; no extension arithmetic).

A workload is cut into consecutive chunks of pairs.  For each chunk two
SHA-256 digests are kept:

* ``inputs``: the generated pairs themselves (lengths, seeds, X, then the
  base codes of both reads, pair by pair), so that a change of the generator
  is caught before any result is compared;
* ``results``: the eleven integer result fields of every pair, widened to
  int64 little-endian, field-major in ``FIELDS`` order.

The stored digests (``golden/config_digests.json``) are written from the CPU
oracle by ``golden/make_config_digests.py``; the GPU tests hash the library's
results the same way and compare chunk by chunk.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
          "b_begin", "b_end", "left_cells", "right_cells", "status"]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DIGEST_FILE = os.path.join(GOLDEN, "config_digests.json")

# pairs per chunk: ultralong pairs cost up to ~3e9 cells each, so its chunks
# are small enough for the oracle to re-run one when a digest differs
CHUNK = {"plain1k": 1000, "batch10k": 1000, "uneven": 1000, "ultralong": 10}


def input_digest(bt) -> str:
    h = hashlib.sha256()
    for p in range(bt.n):
        hdr = np.array([bt.a_len[p], bt.b_len[p], bt.a_seed[p], bt.b_seed[p], bt.x[p], bt.k],
                       dtype="<i8")
        h.update(hdr.tobytes())
        a, b = bt.pair(p)
        h.update(np.ascontiguousarray(a, dtype=np.uint8).tobytes())
        h.update(np.ascontiguousarray(b, dtype=np.uint8).tobytes())
    return h.hexdigest()


def result_digest(res, lo: int = 0, hi: int = None) -> str:
    """Digest of result rows [lo, hi) of a structured array with FIELDS."""
    hi = len(res) if hi is None else hi
    h = hashlib.sha256()
    for f in FIELDS:
        h.update(np.ascontiguousarray(res[f][lo:hi], dtype="<i8").tobytes())
    return h.hexdigest()


def chunks(n: int, size: int):
    return [(lo, min(lo + size, n)) for lo in range(0, n, size)]


def load():
    with open(DIGEST_FILE) as f:
        return json.load(f)


def _generate_chunk(args):
    workload, lo, hi = args
    from paper_2002_05200_amd import synth
    bt = synth.make_batch(workload, n=hi - lo, start=lo)
    return lo, input_digest(bt), bt


def generate(workload: str, workers: int = 1):
    """The whole workload, generated chunk by chunk (in a fork pool when
    workers > 1), and the input digest of every chunk."""
    from paper_2002_05200_amd import synth
    n = synth.WORKLOADS[workload].n_pairs
    args = [(workload, lo, hi) for lo, hi in chunks(n, CHUNK[workload])]
    if workers > 1:
        got = synth.pool_map(_generate_chunk, args, workers)
    else:
        got = [_generate_chunk(a) for a in args]
    got.sort(key=lambda g: g[0])
    return synth.concat([g[2] for g in got], name=workload), [g[1] for g in got]
