"""Benchmark: batched X-drop seed extension on one MI355X.

One step = one xdrop_extend call over the whole workload (planning, every
lane-width tier, the global-memory tier, combining), inputs resident in HBM.
Default workload: 100,000 read pairs, |A| log-normal (median 10 kb), 15% error,
X = 50, scores +1/-1/-1, 17-mer seeds (seeded synthetic data).

Prints one JSON line.  `value` is GCUPS = cells computed / second, cells as
the oracle counts them (every cell of every computed anti-diagonal range).
`roofline` prices the dominant kernel against the INT32 VALU peak at 9
algorithmic int32 operations per cell, with that kernel's duration taken from
HIP events recorded by the library around it on the launch stream.
`sched_compare` runs the other scheduler (the plain one-wavefront-per-job
grid against the persistent queue) on the same resident inputs;
`host_buffers` times the host-memory entry point (allocation, PCIe copies
both ways and the step) on the same reads.  `other_workloads` times the
plain 1 kb, uneven and ultra-long batches whole with the autotuner's options
(uneven and plain1k also with the plain grids, on the same resident inputs)
and checks every pair against the oracle's stored digests.  `seed_choice`
times the GPU seed choice (xd_find_seeds) over the same resident reads and
checks a sample against the seed oracle.  `serving` is the
continuous-batching server under Poisson arrivals at a fraction of its
saturation rate, with a sweep over further loads.  `cpu_baseline` times the
CPU oracle, single-threaded, on an evenly spread sample of the same workload,
and once more with one process per host core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The serving leg runs several slots, each on its own stream; HIP maps streams
# onto GPU_MAX_HW_QUEUES hardware queues (4 unless set), and streams sharing a
# queue run their kernels one after another.  Set before the runtime starts
# (an environment that already fixes a smaller number is raised to 16).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "GCUPS (computed cells) at 1 MI355X, % INT32 roofline; p50/p99 latency in serving"
OPS_PER_CELL = 9                       # algorithmic int32 operations per cell
N_CU, LANES, CLOCK_HZ = 256, 64, 2.4e9
INT32_PEAK_TOPS = N_CU * LANES * CLOCK_HZ / 1e12   # 39.32 T int32 lane-ops/s


def profiled_traffic(kernel_tag: str, workload: str):
    """HBM bytes per launch of a kernel from its committed counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None, None
    fields = dict(l.split(None, 1) for l in open(path).read().splitlines()
                  if l.startswith(("TRAFFIC_BYTES ", "SOURCE_SHA256 ")))
    from paper_2002_05200_amd import build as lib_build
    if fields.get("SOURCE_SHA256", "").strip() != lib_build.source_hash():
        return None, os.path.relpath(path, ROOT) + " (stale: sources changed)"
    return int(fields["TRAFFIC_BYTES"]), os.path.relpath(path, ROOT)


def host_cpu() -> dict:
    """The host the CPU baseline ran on: logical CPUs, those this process may
    use, and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(workload: str, budget_s: float, n_total: int, gpu_results=None) -> dict:
    from oracle import oracle
    from paper_2002_05200_amd import synth
    # grow an evenly spread sample until the oracle has run for about budget_s
    n = 16
    cells = 0
    secs = 0.0
    used = 0
    while secs < budget_s and used < n_total:
        stride = max(1, n_total // max(n, 1))
        bt = synth.make_batch(workload, n=n, start=used % max(stride, 1), stride=stride)
        res, t = oracle.batch(bt, return_time=True)
        cells += int(res["left_cells"].sum() + res["right_cells"].sum())
        secs += t
        used += n
        n *= 2
    return {"value": round(cells / secs / 1e9, 4), "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": f"{used} pairs of the same workload spread evenly over it "
                      f"({cells} cells, {secs:.1f} s, one thread)",
            "host": host_cpu(),
            "all_cores": cpu_all_cores(workload, n_total, used, gpu_results)}


def eq1_ceiling(workload: str, n_total: int, tier: int, n_sample: int = 400) -> dict:
    """Adapted lane-occupancy ceiling (Section VII, Eq. 1) of one tier: the
    oracle traces the computed range of every anti-diagonal of an evenly
    spread sample of pairs (both extensions of each), and each anti-diagonal
    is priced at the lanes the tier that computes it issues."""
    from oracle import oracle
    from paper_2002_05200_amd import ceiling, synth
    n = min(n_sample, n_total)
    stride = max(1, n_total // n)
    bt = synth.make_batch(workload, n=n, start=0, stride=stride)
    m_, mm, g = bt.scores
    jobs = []
    for p in range(bt.n):
        a, b = bt.pair(p)
        pa, pb, k, x = int(bt.a_seed[p]), int(bt.b_seed[p]), bt.k, int(bt.x[p])
        for ea, eb in ((a[:pa][::-1], b[:pb][::-1]), (a[pa + k:], b[pb + k:])):
            tr = oracle.extend(ea, eb, m_, mm, g, x=x, trace=True)["trace"]
            jobs.append(((tr["hi"] - tr["lo"] + 1).tolist(),
                         ceiling.initial_tier(len(ea), len(eb), x)))
    c = ceiling.ceiling(jobs, only_tier=tier)
    return {"frac": round(c["work_weighted"], 4), "eq1_mean": round(c["eq1_mean"], 4),
            "tier": tier, "anti_diagonals": c["anti_diagonals"],
            "sample": f"{bt.n} pairs spread evenly over the workload (both extensions), "
                      f"widths from the oracle's per-anti-diagonal trace",
            "lanes_model": "64 lanes per anti-diagonal with one register, 128 with two, "
                           "the spanned registers with more"}


RESULT_FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
                 "b_begin", "b_end", "left_cells", "right_cells", "status"]


def _oracle_shard(args):
    workload, n_total, start, stride, n = args
    from oracle import oracle
    from paper_2002_05200_amd import synth
    bt = synth.make_batch(workload, n=n, start=start, stride=stride)
    res, t = oracle.batch(bt, return_time=True)
    idx = start + stride * np.arange(n, dtype=np.int64)
    fields = np.stack([res[f] for f in RESULT_FIELDS], axis=1)
    return int(res["left_cells"].sum() + res["right_cells"].sum()), t, idx, fields


def cpu_all_cores(workload: str, n_total: int, n_sample: int, gpu_results=None) -> dict:
    """The same oracle, one process per usable host CPU (at most 16), each on
    its own evenly spread shard as large as the single-thread sample (fewer
    pairs when the workload runs out); GCUPS = all cells / the slowest shard's
    time.  When the shards cover pairs of the timed GPU run, every integer
    result field of those pairs is compared with the GPU's."""
    procs = max(1, min(16, host_cpu()["usable_cpus"]))
    per = max(1, min(n_sample, n_total // procs))
    stride = max(1, n_total // (per * procs))
    jobs = [(workload, n_total, p, stride * procs, per) for p in range(procs)]
    from paper_2002_05200_amd import synth
    out = synth.pool_map(_oracle_shard, jobs, procs)
    cells = sum(o[0] for o in out)
    slowest = max(o[1] for o in out)
    rec = {"value": round(cells / slowest / 1e9, 4), "unit": "GCUPS", "cores": procs,
           "sample": f"{per * procs} pairs in {procs} shards ({cells} cells, slowest shard "
                     f"{slowest:.1f} s)"}
    if gpu_results is not None:
        idx = np.concatenate([o[2] for o in out])
        ref = np.concatenate([o[3] for o in out])
        got = np.stack([gpu_results[f][idx].astype(np.int64) for f in RESULT_FIELDS], axis=1)
        bad = np.nonzero((got != ref).any(axis=1))[0]
        rec["gpu_parity"] = {"pairs_compared": int(len(idx)), "fields": len(RESULT_FIELDS),
                             "mismatched_pairs": int(len(bad)),
                             "first_mismatches": idx[bad[:5]].tolist()}
    return rec


def serving_leg(n_distinct: int, n_requests: int, load: float, slots: int, max_batch: int,
                graph: bool, workers: int, sweep=(), sweep_requests: int = 0,
                sched: str = "plain", by_class: bool = True) -> dict:
    """Continuous-batching serving run: saturation throughput closed-loop (whose
    requests are also the warm-up), then Poisson arrivals at load * saturation;
    latency from the scheduled arrival to the completion the server's
    scheduler observed (same steady clock).  `sweep` repeats the open-loop run
    at other loads with sweep_requests requests each."""
    import threading
    from paper_2002_05200_amd import synth, xdrop
    t0 = time.time()
    if workers > 1:
        reqs = synth.pool_map(synth.make_request, range(n_distinct), workers, chunksize=8)
    else:
        reqs = [synth.make_request(r) for r in range(n_distinct)]
    packed = [xdrop.PackedRequest(bt) for bt in reqs]
    print(f"[bench] serving: {n_distinct} distinct requests generated in {time.time()-t0:.1f} s",
          file=sys.stderr, flush=True)
    sched_code = {"auto": xdrop.SCHED_AUTO, "plain": xdrop.SCHED_PLAIN,
                  "persistent": xdrop.SCHED_PERSISTENT}[sched]
    srv = xdrop.Server(slots=slots, max_batch_pairs=max_batch, graph=int(graph),
                       mem_budget=2 << 30, opts=xdrop.make_opts(sched=sched_code),
                       group_by_class=int(by_class))
    try:
        def closed(n):
            ts = [srv.submit(packed[i % n_distinct]) for i in range(n)]
            cells = 0
            for i, t in enumerate(ts):
                r, _ = srv.poll(t, packed[i % n_distinct].n, wait_ms=-1)
                cells += int(r["left_cells"].sum() + r["right_cells"].sum())
            return cells
        n_sat = 3 * n_distinct             # long enough that ramp-up and drain are small
        # warm-up: one untimed pass of the same closed loop, so every slot has
        # captured its graph and run batches of every class before the timing
        # (with 200 warm-up requests the first measurement ran about a quarter
        # below the steady rate)
        closed(n_sat)
        t1 = time.perf_counter()
        sat_cells = closed(n_sat)
        sat_s = time.perf_counter() - t1
        r_sat = n_sat / sat_s
        sat_gcups = sat_cells / sat_s / 1e9

        def open_loop(load, n_requests, seed_key):
            rate = load * r_sat
            arrivals = synth.poisson_arrivals(n_requests, rate, seed_key)
            tickets = [None] * n_requests
            sched_ns = [0] * n_requests
            lat = np.zeros(n_requests)
            cells = np.zeros(n_requests)
            done_ns = np.zeros(n_requests, np.int64)
            ready = threading.Semaphore(0)

            def poller():
                for i in range(n_requests):
                    ready.acquire()
                    r, dn = srv.poll(tickets[i], packed[i % n_distinct].n, wait_ms=-1)
                    lat[i] = (dn - sched_ns[i]) / 1e6
                    done_ns[i] = dn
                    cells[i] = int(r["left_cells"].sum() + r["right_cells"].sum())

            th = threading.Thread(target=poller)
            th.start()
            start = time.monotonic_ns() + 2_000_000
            for i in range(n_requests):
                sched_ns[i] = start + int(arrivals[i] * 1e9)
                while time.monotonic_ns() < sched_ns[i]:
                    pass
                tickets[i] = srv.submit(packed[i % n_distinct])
                ready.release()
            th.join()
            window = (done_ns.max() - start) / 1e9
            return {"load": load, "requests": n_requests, "rate_requests_per_s": round(rate, 1),
                    "p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "gcups": round(float(cells.sum()) / window / 1e9, 2)}

        main_run = open_loop(load, n_requests, 0)
        print(f"[bench] serving at load {load}: {main_run}", file=sys.stderr, flush=True)
        others = []
        for k, ld in enumerate(sweep):
            others.append(open_loop(ld, sweep_requests, k + 1))
            print(f"[bench] serving at load {ld}: {others[-1]}", file=sys.stderr, flush=True)
        st = srv.stats()
    finally:
        srv.close()
    out = {"requests": n_requests, "warmup_requests": 2 * n_sat,
           "distinct_requests": n_distinct, "saturation_requests_per_s": round(r_sat, 1),
           "saturation_gcups": round(sat_gcups, 2), "saturation_requests": n_sat}
    out.update(main_run)
    out.update({"slots": slots, "max_batch_pairs": max_batch, "graph": bool(graph),
                "batch_sched": sched, "group_by_class": bool(by_class),
                "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                "device_bytes": st["device_bytes"], "mem_budget": 2 << 30,
                "batches": st["batches"], "max_inflight": st["max_inflight"],
                "load_sweep": others, "workload": synth.WORKLOADS["serving"].describe})
    return out


def sched_compare(ctx, db, stream, args, tuned, gcups, ref) -> dict:
    """The other scheduler (plain one-wavefront-per-job grid, or the persistent
    queue) on the same resident inputs, with identical results required."""
    import torch
    from paper_2002_05200_amd import xdrop
    other = "persistent" if args.sched == "plain" else "plain"
    code = xdrop.SCHED_PERSISTENT if other == "persistent" else xdrop.SCHED_PLAIN
    o = xdrop.make_opts(sched=code, **tuned)
    steps = max(2, args.steps // 5)
    ctx.extend_device(db, stream=stream, opts=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.extend_device(db, stream=stream, opts=o)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = db.results()
    assert all(np.array_equal(res[f], ref[f]) for f in ref.dtype.names), \
        f"{other} results differ from {args.sched}"
    cells = int(res["left_cells"].sum() + res["right_cells"].sum())
    mine = "persistent" if args.sched == "auto" else args.sched
    return {mine: round(gcups, 2), other: round(cells * steps / el / 1e9, 2),
            f"{other}_steps": steps, "results_identical": True}


def host_buffers(ctx, db, args, tuned, cells_per_step, ref) -> dict:
    """xdrop_extend_host on the same packed reads and pair records held in host
    memory: device allocation, copies in over PCIe, the step, results back."""
    from paper_2002_05200_amd import xdrop
    sched = {"auto": xdrop.SCHED_AUTO, "plain": xdrop.SCHED_PLAIN,
             "persistent": xdrop.SCHED_PERSISTENT}[args.sched]
    o = xdrop.make_opts(sched=sched, **tuned)
    ctx.extend_host_packed(db.a_words, db.b_words, db.pairs, db.scores, o)
    times = []
    for _ in range(2):
        t0 = time.perf_counter()
        out = ctx.extend_host_packed(db.a_words, db.b_words, db.pairs, db.scores, o)
        times.append(time.perf_counter() - t0)
    assert all(np.array_equal(out[f], ref[f]) for f in ref.dtype.names), "host path differs"
    ms = min(times) * 1e3
    mb_in = (db.a_words.nbytes + db.b_words.nbytes + db.pairs.nbytes) / 1e6
    return {"api": "xdrop_extend_host", "ms_per_call": round(ms, 3),
            "gcups": round(cells_per_step / (ms / 1e3) / 1e9, 2), "mb_in": round(mb_in, 1),
            "mb_out": round(len(out) * out.dtype.itemsize / 1e6, 1),
            "note": "pageable host buffers; includes device allocation and both copies"}


def kernel_name(tier: int, multi_wave: int):
    """Name and file tag of the kernel that runs a tier (stage) of the step."""
    if tier >= 6:   # the stage after the register tiers: a workgroup per job, then HBM
        return ("k_extend_mw<4, 16> + k_spill (bands wider than 2,048 slots: 4 wavefronts "
                "per job, then a global-memory band)", "k_extend_huge")
    c = 1 << tier
    if tier >= 3 and multi_wave in (1, 2):
        nw = 4 if multi_wave == 1 else 2
        return (f"k_extend_mw<{nw}, {c // nw}> ({nw} wavefronts per job, {c} cells per lane "
                f"in all)", f"k_extend_mw{nw}{c // nw}")
    return f"k_extend<C={c}> (cells per lane {c})", f"k_extend_c{c}"


def dominant_kernel(ctx, db, opts_kw: dict) -> dict:
    """One profiled step (HIP events around every stage on the launch stream):
    the stage that takes longest, priced against the INT32 roofline."""
    import torch
    from paper_2002_05200_amd import xdrop
    ctx.extend_device(db, opts=xdrop.make_opts(profile=1, **{k: v for k, v in opts_kw.items()
                                                             if k != "graph"}))
    st = ctx.stats()
    torch.cuda.synchronize()
    tiers_ms = st["stage_ms"][1:8]
    dom = int(np.argmax(tiers_ms))
    cells = int(st["cells"][dom])
    ms = float(tiers_ms[dom])
    name, _ = kernel_name(dom, opts_kw.get("multi_wave", 0))
    achieved = cells * OPS_PER_CELL / (ms / 1e3) / 1e12
    return {"kernel": name, "ms": round(ms, 3), "cells": cells,
            "frac": round(achieved / INT32_PEAK_TOPS, 4),
            "stage_ms": {k: round(float(v), 3) for k, v in zip(
                ["plan", "tier0", "tier1", "tier2", "tier3", "tier4", "tier5", "spill",
                 "combine"], st["stage_ms"])}}


def seed_leg(ctx, db, steps: int, k: int = 17, width: int = 500):
    """xd_find_seeds over the same resident reads (every pair's k-mer matches
    binned by diagonal), timed with HIP events on its stream.  Returns the
    record and the seeds (checked against the seed oracle in the CPU leg)."""
    import torch
    from paper_2002_05200_amd import xdrop
    stream = torch.cuda.current_stream()
    d_seeds = ctx.find_seeds_device(db, k=k, width=width)          # warm-up
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        ctx.find_seeds_device(db, k=k, width=width, d_seeds=d_seeds)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    got = d_seeds[: db.n * xdrop.SEED_DTYPE.itemsize].cpu().numpy().view(xdrop.SEED_DTYPE).copy()
    kmers = int(np.maximum(db.pairs["a_len"].astype(np.int64) - k + 1, 0).sum() +
                np.maximum(db.pairs["b_len"].astype(np.int64) - k + 1, 0).sum())
    bases = int(db.pairs["a_len"].astype(np.int64).sum() + db.pairs["b_len"].astype(np.int64).sum())
    rec = {"api": "xd_find_seeds", "k": k, "width": width, "steps": steps,
           "ms_per_call": round(ms, 3), "pairs_per_s": round(db.n / (ms / 1e3), 1),
           "gkmers_per_s": round(kmers / (ms / 1e3) / 1e9, 3),
           "packed_bases_gb_per_s": round(bases / 4 / (ms / 1e3) / 1e9, 2),
           "found": int((got["found"] == 1).sum()), "pairs": db.n,
           "matches_total": int(got["matches"].sum())}
    return rec, got


def seed_oracle_check(workload: str, gpu_seeds, n_check: int = 2000, k: int = 17,
                      width: int = 500) -> dict:
    """The seed oracle on an evenly spread sample of the workload's pairs,
    compared field by field with the GPU's seeds of those pairs."""
    from oracle import oracle
    from paper_2002_05200_amd import synth
    n = len(gpu_seeds)
    stride = max(1, n // n_check)
    idx = np.arange(0, n, stride)[:n_check]
    bt = synth.make_batch(workload, n=len(idx), start=0, stride=stride)
    t0 = time.perf_counter()
    ref = oracle.find_seeds(bt, k=k, width=width)
    secs = time.perf_counter() - t0
    fields = ["a_seed", "b_seed", "bin_matches", "matches", "found", "status"]
    bad = [int(i) for j, i in enumerate(idx)
           if any(int(gpu_seeds[f][i]) != int(ref[f][j]) for f in fields)]
    return {"pairs_compared": len(idx), "mismatched_pairs": len(bad), "first": bad[:5],
            "sample": f"every {stride}th pair", "oracle_s": round(secs, 2),
            "oracle_pairs_per_s_one_thread": round(len(idx) / secs, 1)}


def workload_leg(name: str, steps: int, plain: bool, workers: int) -> dict:
    """Another batch workload timed whole with the autotuner's options (and,
    with `plain`, with the plain one-wavefront-per-job grids on the same
    resident inputs); every pair's eleven result fields are checked against
    the oracle's stored per-chunk digests."""
    import torch
    from paper_2002_05200_amd import synth, tune, xdrop
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import digests
    t0 = time.time()
    bt, _ = digests.generate(name, workers)
    gen_s = time.time() - t0
    tuned = tune.lookup(bt) or {}
    db = xdrop.DeviceBatch(bt, "cuda:0")
    del bt
    ctx = xdrop.Context(0)
    golden = digests.load()["workloads"].get(name)
    if name == "plain1k":           # sub-millisecond steps: time many
        steps = max(steps, 50)
    out = {"workload": synth.WORKLOADS[name].describe, "pairs": db.n,
           "generate_s": round(gen_s, 1)}
    try:
        variants = [("tuned", xdrop.make_opts(**tuned), None)]
        if plain:
            variants.append(("plain", xdrop.make_opts(sched=xdrop.SCHED_PLAIN), None))
        if name == "plain1k":       # a small batch: launches dominate, so replay a graph
            variants.append(("tuned_graph", xdrop.make_opts(graph=1, **tuned),
                             torch.cuda.Stream()))
        ref = None
        for label, o, strm in variants:
            ctx.extend_device(db, opts=o, stream=strm)    # warm-up (and graph capture)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(steps):
                ctx.extend_device(db, opts=o, stream=strm)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t1) / steps
            res = db.results()
            cells = int(res["left_cells"].sum() + res["right_cells"].sum())
            rec = {"ms_per_step": round(el * 1e3, 3), "gcups": round(cells / el / 1e9, 2),
                   "steps": steps, "cells_per_step": cells}
            if label == "tuned":
                rec["options"] = tuned or "defaults"
                st = ctx.stats()
                rec["jobs_per_tier"] = st["jobs"].tolist()
                rec["restarted"] = int(st["restarted"].sum())
                rec["dominant_kernel"] = dominant_kernel(ctx, db, tuned)
            if ref is None:
                ref = res
            else:
                rec["results_identical_to_tuned"] = bool(
                    all(np.array_equal(res[f], ref[f]) for f in RESULT_FIELDS))
            out[label] = rec
            print(f"[bench] {name} {label}: {rec}", file=sys.stderr, flush=True)
        if golden is not None:
            bad = [c["lo"] for c in golden["chunks"]
                   if digests.result_digest(ref, c["lo"], c["hi"]) != c["results"]]
            out["oracle_parity"] = {"pairs_compared": db.n, "chunks": len(golden["chunks"]),
                                    "mismatched_chunks": len(bad), "first": bad[:3],
                                    "how": "per-chunk SHA-256 of all eleven result fields against "
                                           "the oracle's stored digests"}
        else:
            out["oracle_parity"] = None
        if plain:
            out["persistent_over_plain"] = round(out["tuned"]["gcups"] / out["plain"]["gcups"], 3)
    finally:
        ctx.close()
        del db
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch10k")
    ap.add_argument("--pairs", type=int, default=0, help="0 = the whole workload")
    ap.add_argument("--sched", default="auto", choices=["auto", "plain", "persistent"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=20000,
                    help="requests of the serving leg at --serving-load (0 = skip the leg)")
    ap.add_argument("--serving-sweep", default="0.3,0.5,0.9",
                    help="further loads (fractions of saturation) of the serving leg")
    ap.add_argument("--serving-sweep-requests", type=int, default=4000)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other-scheduler and host-buffer legs")
    ap.add_argument("--serving-distinct", type=int, default=1000,
                    help="distinct generated requests the serving leg cycles through")
    ap.add_argument("--serving-load", type=float, default=0.7)
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-sched", default="plain", choices=["auto", "plain", "persistent"],
                    help="launch schedule of each serving batch (small batches: plain grids)")
    ap.add_argument("--serving-by-class", type=int, default=1,
                    help="1 = batches take requests of one cost class only")
    ap.add_argument("--serving-batch", type=int, default=2048)
    ap.add_argument("--serving-graph", type=int, default=1)
    ap.add_argument("--waves-per-cu", type=int, default=None,
                    help="force the persistent grid size (default: tuned table or per tier)")
    ap.add_argument("--multi-wave", type=int, default=None,
                    help="force the multi_wave launch option (default: tuned table or 0)")
    ap.add_argument("--tuned", action="store_true",
                    help="launch options from the autotuner's table for this workload class")
    ap.add_argument("--graph", action="store_true",
                    help="time hipGraph replays of the step (stage times then come from one "
                         "extra profiled eager step)")
    ap.add_argument("--other-workloads", default="plain1k,uneven,ultralong",
                    help="further batch workloads timed whole (tuned options; uneven and "
                         "plain1k also with the plain grids), empty = none")
    ap.add_argument("--other-steps", type=int, default=3)
    ap.add_argument("--seed-steps", type=int, default=5,
                    help="timed xd_find_seeds calls over the batch's reads (0 = skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every extension "
              f"job is independent, so several GPUs would shard the job list without any "
              f"collective. Not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2002_05200_amd import synth, xdrop

    wl = synth.WORKLOADS[args.workload]
    n_pairs = args.pairs or wl.n_pairs
    t0 = time.time()
    bt = synth.make_batch(args.workload, n=n_pairs, workers=min(16, os.cpu_count() or 1))
    print(f"[bench] generated {bt.n} pairs ({bt.total_bases()/1e9:.2f} Gbases) in "
          f"{time.time()-t0:.1f} s", file=sys.stderr, flush=True)
    tuned = {}
    if args.tuned:
        from paper_2002_05200_amd import tune
        tuned = tune.lookup(bt) or {}
        tuned.pop("sched", None)
        print(f"[bench] tuned options for {tune.batch_class(bt)}: {tuned}", file=sys.stderr,
              flush=True)
    if args.multi_wave is not None:
        tuned["multi_wave"] = args.multi_wave
    if args.waves_per_cu is not None:
        tuned["waves_per_cu"] = args.waves_per_cu
    t0 = time.time()
    db = xdrop.DeviceBatch(bt, "cuda:0")
    del bt.a, bt.b
    torch.cuda.synchronize()
    print(f"[bench] packed + uploaded in {time.time()-t0:.1f} s "
          f"({(len(db.a_words)+len(db.b_words))*4/1e6:.0f} MB resident)", file=sys.stderr, flush=True)
    if args.copy_mb:
        src = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = xdrop.Context(0)
    sched = {"auto": xdrop.SCHED_AUTO, "plain": xdrop.SCHED_PLAIN,
             "persistent": xdrop.SCHED_PERSISTENT}[args.sched]
    opts = xdrop.make_opts(sched=sched, profile=1, **tuned)
    stream = torch.cuda.current_stream()
    if args.graph:
        stream = torch.cuda.Stream()
        gopts = xdrop.make_opts(sched=sched, graph=1, **tuned)

    for _ in range(args.warmup):
        ctx.extend_device(db, stream=stream, opts=gopts if args.graph else opts)
    torch.cuda.synchronize()
    res = db.results() if args.warmup else None

    stage_ms = np.zeros(9)
    tier_cells = np.zeros(7)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    if args.graph:
        for _ in range(args.steps):
            ctx.extend_device(db, stream=stream, opts=gopts)
        torch.cuda.synchronize()
    else:
        for _ in range(args.steps):
            ctx.extend_device(db, stream=stream, opts=opts)
            st = ctx.stats()                  # synchronises; reads the step's HIP events
            stage_ms += st["stage_ms"]
            tier_cells += st["cells"]
        torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    if args.graph:                            # stage times of one profiled eager step
        ctx.extend_device(db, stream=stream, opts=opts)
        st = ctx.stats()
        stage_ms += st["stage_ms"] * args.steps
        tier_cells += st["cells"] * args.steps
    res2 = db.results()
    if res is not None:
        assert np.array_equal(res2["score"], res["score"]), "results changed between steps"
    assert (res2["status"] == 0).all(), "pairs failed"
    cells_per_step = int(res2["left_cells"].sum() + res2["right_cells"].sum())

    gcups = cells_per_step * args.steps / elapsed / 1e9
    # dominant kernel: the tier stage with the largest total time
    tiers_ms = stage_ms[1:8]
    dom = int(np.argmax(tiers_ms))
    dom_ms_per_launch = tiers_ms[dom] / args.steps
    dom_cells_per_launch = tier_cells[dom] / args.steps
    achieved = dom_cells_per_launch * OPS_PER_CELL / (dom_ms_per_launch / 1e3) / 1e12
    kname, ktag = kernel_name(dom, tuned.get("multi_wave", 0))
    traffic, traffic_src = profiled_traffic(ktag, args.workload)
    if n_pairs != wl.n_pairs:          # the summary covers the whole workload only
        traffic, traffic_src = None, None
    line = {
        "metric": METRIC,
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.describe}", "pairs": n_pairs,
                   "jobs": 2 * n_pairs, "x": wl.x, "scores": [1, -1, -1], "seed_k": 17,
                   "sched": args.sched, "graph": bool(args.graph), "tuned": tuned or None,
                   "cells_per_step": cells_per_step},
        "roofline": {"bound": "alu", "kernel": kname,
                     "achieved": round(achieved, 3), "peak": round(INT32_PEAK_TOPS, 3),
                     "unit": "TOP/s (int32 lane ops)", "frac": round(achieved / INT32_PEAK_TOPS, 4),
                     "traffic": traffic, "traffic_source": traffic_src,
                     "ops_per_cell": OPS_PER_CELL,
                     "kernel_ms_per_launch": round(dom_ms_per_launch, 4),
                     "kernel_cells_per_launch": int(dom_cells_per_launch),
                     "stage_ms_per_step": {k: round(v / args.steps, 4) for k, v in zip(
                         ["plan", "tier0", "tier1", "tier2", "tier3", "tier4", "tier5", "spill",
                          "combine"], stage_ms)}},
    }
    if not args.no_compare:
        line["sched_compare"] = sched_compare(ctx, db, stream, args, tuned, gcups, res2)
        line["host_buffers"] = host_buffers(ctx, db, args, tuned, cells_per_step, res2)
    gpu_seeds = None
    if args.seed_steps and args.workload == "batch10k" and n_pairs == wl.n_pairs:
        line["seed_choice"], gpu_seeds = seed_leg(ctx, db, args.seed_steps)
        print(f"[bench] seed choice: {line['seed_choice']}", file=sys.stderr, flush=True)
    ctx.close()
    del db
    others = [w.strip() for w in args.other_workloads.split(",") if w.strip()]
    if others:
        line["other_workloads"] = {
            w: workload_leg(w, args.other_steps, w in ("uneven", "plain1k"),
                            min(16, os.cpu_count() or 1)) for w in others}
    if args.serving_requests:
        sweep = [float(v) for v in args.serving_sweep.split(",") if v.strip()]
        line["serving"] = serving_leg(args.serving_distinct, args.serving_requests,
                                      args.serving_load, args.serving_slots, args.serving_batch,
                                      bool(args.serving_graph), min(16, os.cpu_count() or 1),
                                      sweep, args.serving_sweep_requests, args.serving_sched,
                                      bool(args.serving_by_class))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget, n_pairs, res2)
        if gpu_seeds is not None:
            sc = seed_oracle_check(args.workload, gpu_seeds)
            line["cpu_baseline"]["seed_oracle"] = sc
            line["seed_choice"]["oracle_parity"] = {
                k: sc[k] for k in ("pairs_compared", "mismatched_pairs", "first", "sample")}
        if dom < 6:
            ce = eq1_ceiling(args.workload, n_pairs, dom)
            ce["achieved_over_ceiling"] = round(line["roofline"]["frac"] / ce["frac"], 4) \
                if ce["frac"] else None
            line["roofline"]["eq1_ceiling"] = ce
        gp = line["cpu_baseline"]["all_cores"].get("gpu_parity")
        if gp is not None:
            line["oracle_parity"] = {"pairs_compared": gp["pairs_compared"],
                                     "of_pairs": n_pairs, "mismatched_pairs": gp["mismatched_pairs"],
                                     "how": "every integer result field of the timed run against "
                                            "the all-core oracle leg's results"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
