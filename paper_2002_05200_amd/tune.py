"""Autotuner for the batch launch options of libxdrop.

The kernels' results never depend on these options, only their speed does:
- waves_per_cu: size of the persistent grid (waves per compute unit);
- long_job / long_tier_bias: the short/long split (jobs with m + n at least
  long_job start long_tier_bias lane-width tiers wider, so bands that will
  grow wide skip the narrow windows they would outgrow);
- sort_jobs: longest-estimated-job-first order on or off;
- multi_wave: four (1) or two (2) wavefronts per job in the widest
  single-job tiers;
- sched: the persistent queue (0) or the plain grids of one wavefront per job
  (1), which win on small batches whose time is mostly launches.

`tune` times candidates on a sample batch already resident on the device
(coordinate descent from the defaults, median of a few repetitions, timed
with HIP events on the launch stream) and returns the fastest option set.
`TABLE` maps a workload class (X and read-length buckets of the batch) to
tuned options; `lookup` finds the entry for a batch.  The table shipped
here was written by `python -m paper_2002_05200_amd.tune` on an MI355X.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tune_table.json")

# A knob named "a+b" sets several options together.  The persistent grid size
# that suits one wavefront per job differs from the multi-wave one (a
# four-wavefront job needs a grid large enough that the longest jobs, not the
# queue, set the end), so those two are searched jointly.
CANDIDATES: Dict[str, list] = {
    "sched": [0, 1],
    "long_tier_bias": [0, 1, 2, 3],
    "long_job": [2000, 10000, 40000],
    "multi_wave+waves_per_cu": [(m, w) for m in (0, 1, 2) for w in (0, 8, 12, 16, 24)],
    "sort_jobs": [1, 0],
}
DEFAULTS = {"sched": 0, "waves_per_cu": 0, "sort_jobs": 1, "long_job": 0, "long_tier_bias": 0,
            "multi_wave": 0}


def workload_class(x: np.ndarray, a_len: np.ndarray, b_len: np.ndarray) -> str:
    """Class of a batch: median X bucket and median pair length (log2 bucket)."""
    xm = float(np.median(x))
    xb = next((b for b in (16, 64, 256, 1024) if xm <= b), 1 << 30)
    lm = float(np.median(a_len.astype(np.int64) + b_len))
    lb = int(math.log2(max(lm, 1.0)))
    return f"x<={xb}/len~2^{lb}"


def batch_class(bt) -> str:
    return workload_class(bt.x, bt.a_len, bt.b_len)


def load_table(path: str = TABLE_PATH) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(bt, table: Optional[dict] = None) -> Optional[dict]:
    """Tuned option dict for the batch's class, or None."""
    t = load_table() if table is None else table
    e = t.get(batch_class(bt))
    return dict(e["opts"]) if e else None


def time_opts(ctx, db, opts_kw: dict, reps: int = 3) -> float:
    """Median milliseconds of one xdrop_extend with these options."""
    import torch
    from . import xdrop
    s = torch.cuda.current_stream()
    o = xdrop.make_opts(**opts_kw)
    ctx.extend_device(db, stream=s, opts=o)        # warm-up (scratch, code)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ctx.extend_device(db, stream=s, opts=o)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def _set(opts: dict, knob: str, value) -> dict:
    """Copy of opts with the knob (one option, or "a+b" several) set to value."""
    out = dict(opts)
    names = knob.split("+")
    for n, v in zip(names, value if len(names) > 1 else (value,)):
        out[n] = v
    return out


def tune(ctx, db, reps: int = 3, log=None, passes: int = 2, timer=None) -> dict:
    """Coordinate descent over CANDIDATES from DEFAULTS, repeated while a pass
    improves (at most `passes` passes: the knobs interact).  `timer(opts)`
    replaces the GPU timing (for tests)."""
    timer = timer or (lambda o: time_opts(ctx, db, o, reps))
    best = dict(DEFAULTS)
    best_ms = timer(best)
    base_ms = best_ms
    tried = {tuple(sorted(best.items())): best_ms}
    for _ in range(passes):
        start = dict(best)
        for knob, values in CANDIDATES.items():
            for v in values:
                cand = _set(best, knob, v)
                if cand == best:
                    continue
                if cand["long_tier_bias"] == 0 and knob == "long_job":
                    continue                      # the split does nothing without a bias
                if cand["long_tier_bias"] > 0 and cand["long_job"] == 0:
                    cand["long_job"] = CANDIDATES["long_job"][0]
                key = tuple(sorted(cand.items()))
                if key in tried:
                    continue
                if log:
                    log(f"  timing {cand}")
                ms = timer(cand)
                tried[key] = ms
                if log:
                    log(f"  {cand} -> {ms:.2f} ms")
                if ms < best_ms:
                    best, best_ms = cand, ms
        if best == start:
            break
    return {"opts": best, "ms": round(best_ms, 3), "default_ms": round(base_ms, 3),
            "candidates": len(tried)}


def main():
    import argparse
    import torch
    from . import synth, xdrop
    ap = argparse.ArgumentParser(description="tune launch options per workload class")
    ap.add_argument("--workloads", default="batch10k,uneven,ultralong,plain1k")
    ap.add_argument("--pairs", type=int, default=0, help="0 = the whole workload")
    ap.add_argument("--sample", type=int, default=20000,
                    help="tune on an evenly spread sample of this many pairs (0 = all)")
    ap.add_argument("--out", default=TABLE_PATH)
    args = ap.parse_args()
    table = load_table(args.out)
    ctx = xdrop.Context(0)
    for wl in args.workloads.split(","):
        total = args.pairs or synth.WORKLOADS[wl].n_pairs
        if args.sample and args.sample < total:
            bt = synth.make_batch(wl, n=args.sample, stride=total // args.sample)
        else:
            bt = synth.make_batch(wl, n=total, workers=min(16, os.cpu_count() or 1))
        db = xdrop.DeviceBatch(bt, "cuda:0")
        cls = batch_class(bt)
        print(f"[tune] {wl}: class {cls}, {bt.n} pairs", flush=True)
        t0 = time.time()
        res = tune(ctx, db, log=lambda m: print(m, flush=True))
        res["tuned_on"] = f"{wl}, {bt.n} pairs"
        table[cls] = res
        print(f"[tune] {wl}: {res['opts']} {res['ms']} ms (default {res['default_ms']} ms, "
              f"{time.time() - t0:.0f} s)", flush=True)
        del db
        torch.cuda.empty_cache()
    ctx.close()
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"[tune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
