"""Writes config_digests.json: per-chunk digests of every pair of the batch
workloads, with the expected results computed by the CPU oracle only.

    python tests/golden/make_config_digests.py [--workers 8] [workload ...]

For each workload (plain1k, batch10k, uneven, ultralong by default) every
pair is generated from its own seeded stream, hashed (``inputs``), extended
by the oracle (Section III-A X-drop, seed split of Section IV-B), and the
eleven integer result fields are hashed per chunk (``results``); the chunk's
cell total and score total are stored beside them for reading.  Chunks run
in a process pool; nothing here depends on the pool size.  Expect about a
core-hour and a half for all four workloads.
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import digests  # noqa: E402

ORDER = ["plain1k", "batch10k", "uneven", "ultralong"]


def one_chunk(args):
    workload, lo, hi = args
    from oracle import oracle
    from paper_2002_05200_amd import synth
    bt = synth.make_batch(workload, n=hi - lo, start=lo)
    res, secs = oracle.batch(bt, return_time=True)
    return {"lo": lo, "hi": hi, "inputs": digests.input_digest(bt),
            "results": digests.result_digest(res),
            "cells": int(res["left_cells"].sum() + res["right_cells"].sum()),
            "score_sum": int(res["score"].sum()), "oracle_s": round(secs, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("workloads", nargs="*", default=ORDER)
    args = ap.parse_args()
    from oracle import oracle
    from paper_2002_05200_amd import synth
    oracle.build()
    import numpy as np

    out = {}
    if os.path.exists(digests.DIGEST_FILE):
        out = digests.load()
    out["about"] = ("Per-chunk SHA-256 digests of the generated pairs and of the oracle's "
                    "eleven integer result fields (int64 LE, field-major); written by "
                    "tests/golden/make_config_digests.py from oracle/ and the generator only")
    out["fields"] = digests.FIELDS
    out["numpy"] = np.__version__
    work = out.setdefault("workloads", {})
    for wl in args.workloads:
        n = synth.WORKLOADS[wl].n_pairs
        parts = digests.chunks(n, digests.CHUNK[wl])
        t0 = time.time()
        with get_context("fork").Pool(args.workers) as pool:
            got = list(pool.imap_unordered(one_chunk, [(wl, lo, hi) for lo, hi in parts],
                                           chunksize=1))
        got.sort(key=lambda c: c["lo"])
        work[wl] = {"pairs": n, "chunk": digests.CHUNK[wl],
                    "cells": sum(c["cells"] for c in got), "chunks": got}
        print(f"{wl}: {n} pairs, {work[wl]['cells']} cells, {len(got)} chunks, "
              f"{time.time() - t0:.0f} s", flush=True)
        with open(digests.DIGEST_FILE, "w") as f:
            json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
