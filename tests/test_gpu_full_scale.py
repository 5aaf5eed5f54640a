"""Full-scale GPU parity: every pair of the plain1k, batch10k, uneven and
ultralong workloads, against the oracle's stored per-chunk digests.

``golden/config_digests.json`` holds, per chunk of consecutive pairs, a digest
of the generated inputs and a digest of the eleven integer result fields the
CPU oracle computed (``golden/make_config_digests.py``, which calls only the
oracle and the generator).  Each test here regenerates the whole workload,
checks the input digests (a changed generator fails here, not as a parity
error), runs the library on all of it with several launch-option sets --
the defaults, the autotuner's table entry for the workload, and the other
scheduler or wavefront count -- and compares the result digests chunk by
chunk.  Where a chunk differs, the oracle re-runs that chunk's pairs and the
first differing pair and field are reported.
"""
import os

import numpy as np
import pytest

import digests

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, os.cpu_count() or 1))


def option_sets(workload, bt):
    from paper_2002_05200_amd import tune
    tuned = tune.lookup(bt) or {}
    tuned.pop("sched", None)
    sets = [("default", None), ("tuned", tuned)]
    if workload == "ultralong":
        sets.append(("two wavefronts per job", dict(multi_wave=2, waves_per_cu=16)))
    else:
        sets.append(("plain grids", dict(sched=1)))
    return sets


def first_difference(workload, res, chunk):
    """Re-runs one chunk through the oracle; names the first differing pair."""
    from oracle import oracle
    from paper_2002_05200_amd import synth
    lo, hi = chunk["lo"], chunk["hi"]
    bt = synth.make_batch(workload, n=hi - lo, start=lo)
    ref = oracle.batch(bt)
    for p in range(hi - lo):
        for f in digests.FIELDS:
            g, r = int(res[f][lo + p]), int(ref[f][p])
            if g != r:
                return (f"pair {lo + p}: field {f} gpu {g} oracle {r} "
                        f"(|A|={int(bt.a_len[p])}, |B|={int(bt.b_len[p])}, X={int(bt.x[p])})")
    return "the oracle agrees with the GPU on every pair of this chunk: stored digest stale"


def check_workload(workload):
    import torch
    from paper_2002_05200_amd import xdrop
    golden = digests.load()["workloads"][workload]
    print(f"[full-scale] generating {workload}", flush=True)
    bt, got_in = digests.generate(workload, WORKERS)
    want_in = [c["inputs"] for c in golden["chunks"]]
    assert len(got_in) == len(want_in)
    drift = [c["lo"] for c, g in zip(golden["chunks"], got_in) if g != c["inputs"]]
    assert not drift, f"{workload}: generated inputs differ from the stored ones at chunks {drift[:5]}"
    sets = option_sets(workload, bt)
    db = xdrop.DeviceBatch(bt, "cuda:0")
    del bt
    ctx = xdrop.Context(0)
    try:
        for label, kw in sets:
            print(f"[full-scale] {workload}: {label} {kw}", flush=True)
            db.d_out.zero_()
            ctx.extend_device(db, opts=xdrop.make_opts(**kw) if kw is not None else None)
            torch.cuda.synchronize()
            res = db.results()
            st = ctx.stats()
            print(f"[full-scale]   jobs per tier {st['jobs'].tolist()} escalated "
                  f"{st['escalated'].tolist()} restarted {st['restarted'].tolist()}", flush=True)
            bad = [c for c in golden["chunks"]
                   if digests.result_digest(res, c["lo"], c["hi"]) != c["results"]]
            if bad:
                where = first_difference(workload, res, bad[0])
                pytest.fail(f"{workload} ({label}): {len(bad)} of {len(golden['chunks'])} chunks "
                            f"differ from the oracle, first at pairs [{bad[0]['lo']}, "
                            f"{bad[0]['hi']}): {where}")
            cells = int(res["left_cells"].sum() + res["right_cells"].sum())
            assert cells == golden["cells"]
    finally:
        ctx.close()


@pytest.mark.parametrize("workload", ["plain1k", "batch10k", "uneven", "ultralong"])
def test_every_pair_matches_the_oracle(workload):
    if workload not in digests.load()["workloads"]:
        pytest.skip(f"no stored digests for {workload}")
    check_workload(workload)


def test_full_save_pool_restarts_stay_exact():
    """A save pool of a few slots: most escalating jobs find no slot and start
    over in the wider tier; results must not change, and the restarts (with
    the cells they recomputed) are counted."""
    from oracle import oracle
    from paper_2002_05200_amd import synth, xdrop
    bt = synth.concat([synth.random_cases(seed=910, n=120, len_lo=200, len_hi=3000,
                                          x_choices=(30, 60, 100, 200, 400, 700),
                                          spurious_frac=0.7),
                       synth.make_batch("uneven", n=40, start=3, stride=4999)], name="pool")
    ref = oracle.batch(bt)
    ctx = xdrop.Context(0)
    try:
        for slots, kw in [(0, {}), (3, {}), (1, {}), (3, dict(multi_wave=1)), (2, dict(sched=1))]:
            print(f"[full-scale] save pool cap {slots} {kw}", flush=True)
            got = ctx.extend(bt, opts=xdrop.make_opts(max_save_slots=slots, **kw))
            st = ctx.stats()
            for f in digests.FIELDS:
                bad = np.nonzero(got[f].astype(np.int64) != ref[f].astype(np.int64))[0]
                assert len(bad) == 0, f"cap {slots} {kw}: field {f} differs at pairs {bad[:8]}"
            esc, rst = int(st["escalated"][:6].sum()), int(st["restarted"][:6].sum())
            print(f"[full-scale]   escalated {esc} restarted {rst} wasted "
                  f"{int(st['wasted_cells'].sum())}", flush=True)
            assert esc > 20
            if slots == 0:
                assert rst == 0 and int(st["wasted_cells"][:6].sum()) == 0
            else:
                assert rst > 0 and int(st["wasted_cells"][:6].sum()) > 0
    finally:
        ctx.close()
