"""GPU parity: the HIP library against the CPU oracle, bit-exact on every
integer field (scores, the four end coordinates, both cell counts, status).

Every case is seeded.  Sizes: the random cases span several hundred
wavefronts with a ragged tail; the workload cases use the real generators;
the full-size case runs the whole 100,000-pair 10 kb workload in the
configuration the benchmark times and checks sampled pairs one by one plus
invariants on every pair.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
          "b_begin", "b_end", "left_cells", "right_cells", "status"]


@pytest.fixture(scope="module")
def xd():
    from paper_2002_05200_amd import xdrop
    return xdrop


@pytest.fixture(scope="module")
def ctx(xd):
    c = xd.Context(0)
    yield c
    c.close()


def oracle_of(bt):
    from oracle import oracle
    return oracle.batch(bt)


def assert_same(got, ref, label=""):
    for f in FIELDS:
        g = got[f].astype(np.int64)
        r = ref[f].astype(np.int64)
        bad = np.nonzero(g != r)[0]
        assert len(bad) == 0, (f"{label}: field {f} differs at pairs {bad[:10].tolist()} "
                               f"(gpu {g[bad[:5]].tolist()} vs oracle {r[bad[:5]].tolist()})")


def run(ctx, xd, bt, **kw):
    print(f"case {bt.name} n={bt.n} opts={kw}", flush=True)
    return ctx.extend(bt, opts=xd.make_opts(**kw) if kw else None)


# ------------------------------------------------------------ random pairs
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("sched", [1, 2])
def test_random_pairs(ctx, xd, seed, sched):
    from paper_2002_05200_amd import synth
    bt = synth.random_cases(seed=100 + seed, n=301, len_lo=17, len_hi=700,
                            x_choices=(0, 1, 2, 3, 5, 10, 20, 50, 100, 1000))
    assert_same(run(ctx, xd, bt, sched=sched), oracle_of(bt), f"random seed {seed} sched {sched}")


@pytest.mark.parametrize("impl", [0, 1])
def test_hand_scheduled_and_c_loops_agree(ctx, xd, impl):
    """The hand-scheduled one-register loop and the portable C loop give the
    same results, and both equal the oracle."""
    from paper_2002_05200_amd import synth
    bt = synth.concat([synth.random_cases(seed=150, n=200, len_lo=17, len_hi=3000,
                                          x_choices=(0, 1, 2, 5, 10, 20, 30, 50)),
                       synth.make_batch("batch10k", n=40, start=7, stride=2003)], name="impl")
    assert_same(run(ctx, xd, bt, impl=impl), oracle_of(bt), f"impl {impl}")
    assert_same(run(ctx, xd, bt, impl=impl, sched=1), oracle_of(bt), f"impl {impl} plain")


@pytest.mark.parametrize("tier", [1, 2, 3, 4, 5])
def test_every_register_tier(ctx, xd, tier):
    """Forcing every job to start at a wider tier must not change any result."""
    from paper_2002_05200_amd import synth
    bt = synth.random_cases(seed=200 + tier, n=129, len_lo=17, len_hi=500,
                            x_choices=(0, 1, 5, 20, 50, 100))
    assert_same(run(ctx, xd, bt, min_tier=tier), oracle_of(bt), f"min_tier {tier}")


@pytest.mark.parametrize("scores", [(2, -3, -2), (1, -2, -1), (3, -1, -2), (1, 0, -1),
                                    (5, -4, -3), (2, -1, -1), (1, -1, -2)])
def test_score_sets(ctx, xd, scores):
    from paper_2002_05200_amd import synth
    bt = synth.random_cases(seed=300, n=97, len_lo=17, len_hi=400,
                            x_choices=(0, 1, 3, 7, 15, 40, 120), scores=scores)
    assert_same(run(ctx, xd, bt), oracle_of(bt), f"scores {scores}")


# ------------------------------------------------------------ edge cases
def test_degenerate_pairs(ctx, xd):
    """Empty extensions, whole-read seeds, k = 0, X = 0, tiny reads."""
    from paper_2002_05200_amd import synth
    r = np.random.default_rng(5)
    a_l, b_l, pa, pb, xs = [], [], [], [], []
    for _ in range(200):
        L = int(r.integers(0, 40))
        a = r.integers(0, 4, L).astype(np.uint8)
        b = a.copy() if r.random() < 0.5 else r.integers(0, 4, int(r.integers(0, 40))).astype(np.uint8)
        p = int(r.integers(0, min(len(a), len(b)) + 1))
        a_l.append(a); b_l.append(b); pa.append(p); pb.append(p)
        xs.append(int(r.integers(0, 5)))
    bt = synth.from_pairs(a_l, b_l, pa, pb, xs, k=0, name="degenerate")
    assert_same(run(ctx, xd, bt), oracle_of(bt), "degenerate")


def test_unbounded_x_reaches_the_global_memory_tier(ctx, xd):
    """X beyond the score range: nothing is pruned, the band is whole
    anti-diagonals (up to 2,500 cells), wider than every register tier."""
    from paper_2002_05200_amd import synth
    r = np.random.default_rng(6)
    a_l, b_l, pa, pb = [], [], [], []
    for L in (300, 2600, 2700, 5000):
        a = r.integers(0, 4, L).astype(np.uint8)
        b = r.integers(0, 4, L).astype(np.uint8)
        b[L // 2: L // 2 + 17] = a[L // 2: L // 2 + 17]
        a_l.append(a); b_l.append(b); pa.append(L // 2); pb.append(L // 2)
    bt = synth.from_pairs(a_l, b_l, pa, pb, [1 << 20] * 4, name="x_unbounded")
    got = run(ctx, xd, bt)
    assert_same(got, oracle_of(bt), "unbounded X")
    st = ctx.stats()
    assert st["jobs"][6] >= 2, st
    assert st["jobs"].sum() == 2 * bt.n


def test_invalid_and_overflowing_pairs_are_flagged_alone(ctx, xd):
    from paper_2002_05200_amd import synth
    good = synth.random_cases(seed=400, n=20, len_lo=17, len_hi=200)
    pr_ok = oracle_of(good)
    a_l = [good.pair(p)[0] for p in range(good.n)]
    b_l = [good.pair(p)[1] for p in range(good.n)]
    pa, pb, xs = good.a_seed.copy(), good.b_seed.copy(), good.x.copy()
    pa[3] = len(a_l[3]) - 5            # seed runs past the read
    pb[7] = len(b_l[7])                # seed starts at the end
    xs[11] = (1 << 29) + 1             # X beyond the accepted range
    bt = synth.from_pairs(a_l, b_l, pa, pb, xs, name="invalid")
    got = run(ctx, xd, bt)
    assert got["status"][3] == xd.XD_EINVAL
    assert got["status"][7] == xd.XD_EINVAL
    assert got["status"][11] == xd.XD_EINVAL
    others = [p for p in range(good.n) if p not in (3, 7, 11)]
    assert_same(got[others], pr_ok[others], "valid pairs beside invalid ones")
    # the int32 guard: (|A| + |B|) * (|match| + |mismatch| + 2|gap|) + X >= 2^29
    big = synth.from_pairs([a_l[0]], [b_l[0]], [pa[0]], [pb[0]], [(1 << 29) - 10], name="guard")
    assert run(ctx, xd, big)["status"][0] == xd.XD_EOVERFLOW


def test_plain_and_persistent_and_host_api_agree(ctx, xd):
    from paper_2002_05200_amd import synth
    bt = synth.make_batch("uneven", n=64)
    a = run(ctx, xd, bt, sched=1)
    b = run(ctx, xd, bt, sched=2)
    c = ctx.extend_host(bt)
    d = run(ctx, xd, bt, sched=2)          # repeat: deterministic
    for other in (b, c, d):
        assert_same(other, a, "schedules")
    assert_same(a, oracle_of(bt), "uneven sample")


# ------------------------------------------------------------ workloads
def test_workload_plain1k_full(ctx, xd):
    from paper_2002_05200_amd import synth
    bt = synth.make_batch("plain1k")
    assert_same(run(ctx, xd, bt), oracle_of(bt), "plain1k (all 1,000 pairs)")


def test_workload_batch10k_sample(ctx, xd):
    from paper_2002_05200_amd import synth
    bt = synth.make_batch("batch10k", n=50, start=0, stride=1999)
    assert_same(run(ctx, xd, bt), oracle_of(bt), "batch10k sample")


def test_workload_uneven_sample(ctx, xd):
    from paper_2002_05200_amd import synth
    bt = synth.make_batch("uneven", n=60, start=1000, stride=3331)
    assert_same(run(ctx, xd, bt), oracle_of(bt), "uneven sample")


def test_workload_serving_requests(ctx, xd):
    from paper_2002_05200_amd import synth
    bt = synth.concat([synth.make_request(r) for r in range(4)], name="serving[0:4]")
    assert_same(run(ctx, xd, bt), oracle_of(bt), "serving requests")


def test_workload_ultralong_sample(ctx, xd):
    from paper_2002_05200_amd import synth
    bt = synth.make_batch("ultralong", n=2, start=0, stride=997)
    assert_same(run(ctx, xd, bt), oracle_of(bt), "ultralong sample")


def test_full_size_batch10k(ctx, xd):
    """All 100,000 pairs in the benchmark's configuration; 64 pairs spread
    over the batch checked one by one, every pair checked for invariants."""
    from paper_2002_05200_amd import synth
    bt = synth.make_batch("batch10k", workers=8)
    got = run(ctx, xd, bt)
    assert (got["status"] == 0).all()
    assert (got["seed_score"] == bt.k).all()
    assert (got["score"] == got["left_score"] + got["seed_score"] + got["right_score"]).all()
    assert (got["left_score"] >= 0).all() and (got["right_score"] >= 0).all()
    assert (got["a_begin"] <= bt.a_seed).all() and (got["a_end"] <= bt.a_len).all()
    assert (got["b_begin"] <= bt.b_seed).all() and (got["b_end"] <= bt.b_len).all()
    # a left job is empty only when the seed starts one of the reads
    nonempty_left = (bt.a_seed > 0) | (bt.b_seed > 0)
    assert (got["left_cells"][nonempty_left] > 0).all()
    assert (got["left_cells"][~nonempty_left] == 0).all()
    idx = np.linspace(0, bt.n - 1, 64).astype(np.int64)
    sub = bt.subset(idx)
    assert_same(got[idx], oracle_of(sub), "batch10k full-size, sampled pairs")


# ------------------------------------------------------------ batch execution
def test_launch_options_do_not_change_results(ctx, xd):
    """Unsorted order, long jobs started wider, other persistent grid sizes:
    same results as the oracle."""
    from paper_2002_05200_amd import synth
    bt = synth.concat([synth.random_cases(seed=500, n=150, len_lo=17, len_hi=2500,
                                          x_choices=(0, 3, 10, 50, 100, 300)),
                       synth.make_batch("uneven", n=24, start=5, stride=7919)], name="opts")
    ref = oracle_of(bt)
    for kw in [dict(sort_jobs=0), dict(long_job=1000, long_tier_bias=2),
               dict(long_job=1, long_tier_bias=5), dict(waves_per_cu=4),
               dict(sched=1, long_job=500, long_tier_bias=1), dict(multi_wave=1),
               dict(multi_wave=1, sched=1), dict(multi_wave=1, min_tier=3),
               dict(multi_wave=2), dict(multi_wave=2, min_tier=3)]:
        assert_same(run(ctx, xd, bt, **kw), ref, f"opts {kw}")


def test_graph_replays_match_eager(ctx, xd):
    """Graph mode: the captured launch sequence replayed several times, with
    eager calls and other device work between the replays, and once more
    after the pair records changed in place (same buffers, new X)."""
    import torch
    from paper_2002_05200_amd import synth
    bt = synth.concat([synth.random_cases(seed=600, n=200, len_lo=17, len_hi=1500,
                                          x_choices=(0, 2, 10, 50, 200)),
                       synth.make_batch("batch10k", n=16, start=3, stride=4001)], name="graph")
    ref = oracle_of(bt)
    db = xd.DeviceBatch(bt, "cuda:0")
    s = torch.cuda.Stream()
    eager = xd.make_opts()
    graph = xd.make_opts(graph=1)
    noise = torch.ones(1 << 20, device="cuda:0")
    for rep in range(4):
        print(f"graph replay {rep}", flush=True)
        db.d_out.zero_()
        ctx.extend_device(db, stream=s, opts=graph)
        s.synchronize()
        assert_same(db.results(), ref, f"graph replay {rep}")
        ctx.extend_device(db, opts=eager)          # eager call on another stream between
        noise.mul_(1.0001).sum().item()
        torch.cuda.synchronize()
        assert_same(db.results(), ref, f"eager after replay {rep}")
    # same buffers, new contents: X of every pair changed
    bt2 = synth.from_pairs([bt.pair(p)[0] for p in range(bt.n)], [bt.pair(p)[1] for p in range(bt.n)],
                           bt.a_seed, bt.b_seed, (bt.x * 2 + 1) % 301, name="graph-x")
    ref2 = oracle_of(bt2)
    pr = xd.make_pairs(bt2)
    db.d_pairs.copy_(torch.from_numpy(pr.view(np.uint8).reshape(-1)))
    torch.cuda.synchronize()
    ctx.extend_device(db, stream=s, opts=graph)
    s.synchronize()
    assert_same(db.results(), ref2, "graph replay after the pairs changed")


@pytest.mark.parametrize("scores", [(1, -1, -1), (2, -3, -2)])
def test_escalated_jobs_resume_in_the_wider_tier(ctx, xd, scores):
    """Bands that outgrow several windows in a row (mostly unrelated reads,
    X up to 700): each escalation hands its state to the next tier, and the
    results still equal the oracle's."""
    from paper_2002_05200_amd import synth
    bt = synth.random_cases(seed=910, n=120, len_lo=200, len_hi=3000,
                            x_choices=(30, 60, 100, 200, 400, 700), spurious_frac=0.7,
                            scores=scores)
    got = run(ctx, xd, bt)
    st = ctx.stats()
    assert st["escalated"][:5].sum() > 20, st
    assert_same(got, oracle_of(bt), f"escalations {scores}")
    assert_same(run(ctx, xd, bt, impl=1), got, "escalations, C loops")
    assert_same(run(ctx, xd, bt, multi_wave=1), got, "escalations, four wavefronts per job")
    assert_same(run(ctx, xd, bt, multi_wave=2), got, "escalations, two wavefronts per job")


def asymmetric_cases(seed, n=150):
    """Pairs whose reads differ in length and content in every way the
    band bookkeeping meets near read ends: noisy copies cut short or
    extended by random tails, unrelated reads, X from 1 to 79."""
    from paper_2002_05200_amd import synth
    r = np.random.default_rng(seed)
    a_l, b_l, pa, pb, xs = [], [], [], [], []
    for _ in range(n):
        a = r.integers(0, 4, int(r.integers(20, 1600))).astype(np.uint8)
        if r.random() < 0.7:
            e = r.uniform(0.02, 0.2) / 3
            b = synth.mutate(r, a, e, e, e)
            if r.random() < 0.5:
                b = b[: int(len(b) * r.uniform(0.3, 1.0))]
            else:
                b = np.concatenate([b, r.integers(0, 4, int(r.integers(0, 800))).astype(np.uint8)])
        else:
            b = r.integers(0, 4, int(r.integers(20, 1600))).astype(np.uint8)
        if len(b) < 17:
            b = np.concatenate([b, r.integers(0, 4, 17).astype(np.uint8)])
        p = int(r.integers(0, len(a) - 16))
        q = int(r.integers(0, len(b) - 16))
        b[q:q + 17] = a[p:p + 17]
        a_l.append(a); b_l.append(b); pa.append(p); pb.append(q); xs.append(int(r.integers(1, 80)))
    return synth.from_pairs(a_l, b_l, pa, pb, xs, name=f"asymmetric{seed}")


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_asymmetric_reads(ctx, xd, seed):
    """Regression: after the hand-scheduled loop left a block, the matrix-
    clipping loop reused score words built for an older window base."""
    bt = asymmetric_cases(seed)
    assert_same(run(ctx, xd, bt), oracle_of(bt), f"asymmetric seed {seed}")


def test_score_words_follow_the_window_after_a_recentre(ctx, xd):
    """Regression for the same bug on the pair that exposed it: a 192 x 443
    right extension at X = 21 that recentres and then reaches the end of A."""
    from paper_2002_05200_amd import synth
    bt = synth.random_cases(seed=600, n=200, len_lo=17, len_hi=1500, x_choices=(0, 2, 10, 50, 200))
    a, b = bt.pair(196)
    one = synth.from_pairs([a], [b], [int(bt.a_seed[196])], [int(bt.b_seed[196])], [21], name="p196")
    assert_same(run(ctx, xd, one), oracle_of(one), "pair 196, X = 21")


def test_bands_wider_than_the_first_spill_pass(ctx, xd):
    """Unbounded X on 40 kb unrelated reads seeded in the middle: anti-
    diagonals reach 20,000 cells, more than the first global-memory pass
    holds, so the job moves to the second pass and starts over there."""
    from paper_2002_05200_amd import synth
    r = np.random.default_rng(7)
    L = 40000
    a = r.integers(0, 4, L).astype(np.uint8)
    b = r.integers(0, 4, L).astype(np.uint8)
    b[L // 2: L // 2 + 17] = a[L // 2: L // 2 + 17]
    bt = synth.from_pairs([a], [b], [L // 2], [L // 2], [1 << 20], name="x_unbounded_40k")
    got = run(ctx, xd, bt)
    st = ctx.stats()
    assert st["escalated"][6] == 2, st
    assert st["jobs"][6] == 2, st
    assert_same(got, oracle_of(bt), "second spill pass")


def test_multi_wave_tier_from_the_start(ctx, xd):
    """Every job straight to the workgroup-per-job tier (4 wavefronts of 16
    registers, 4,096 slots): narrow and wide bands, recentring across
    wavefronts."""
    from paper_2002_05200_amd import synth
    bt = synth.concat([synth.random_cases(seed=700, n=60, len_lo=17, len_hi=900,
                                          x_choices=(0, 1, 5, 20, 100)),
                       synth.make_batch("uneven", n=6, start=11, stride=20011)], name="mw")
    got = run(ctx, xd, bt, min_tier=6)
    st = ctx.stats()
    assert st["jobs"][6] == 2 * bt.n, st
    assert_same(got, oracle_of(bt), "multi-wave tier")


def _ending_pairs(seed, n=48):
    """Pairs whose overlap stops partway: B copies A with 3% of each error
    kind up to a cut and is unrelated after it, so X-drop ends inside the
    reads with the band still wide (X 60-100)."""
    from paper_2002_05200_amd import synth
    rng = np.random.default_rng(np.random.SeedSequence(977, spawn_key=(seed,)))
    a_l, b_l, pa_l, x_l = [], [], [], []
    for _ in range(n):
        la = int(rng.integers(1500, 6000))
        cut = int(rng.integers(300, la - 300))
        a = rng.integers(0, 4, la).astype(np.uint8)
        b = np.concatenate([synth.mutate(rng, a[:cut], 0.03, 0.03, 0.03),
                            rng.integers(0, 4, la - cut).astype(np.uint8)])
        pa = int(rng.integers(0, max(1, min(cut, len(b)) - 17)))
        b[pa:pa + 17] = a[pa:pa + 17]
        a_l.append(a); b_l.append(b); pa_l.append(pa); x_l.append(int(rng.choice([60, 80, 100])))
    return synth.from_pairs(a_l, b_l, pa_l, pa_l, x_l, name=f"ending[{seed}]")


def _edge_riding_pairs(seed, n=24):
    """Pairs of very unequal lengths: one read is a mutated stretch of the
    other (or an unrelated read sharing only the seed) and ends long before
    it, so once it runs out the band keeps going along the matrix edge (j = n
    or i = m) with its range clipped there (X 100-400: bands of hundreds of
    cells)."""
    from paper_2002_05200_amd import synth
    rng = np.random.default_rng(np.random.SeedSequence(1409, spawn_key=(seed,)))
    a_l, b_l, pa_l, pb_l, x_l = [], [], [], [], []
    for t in range(n):
        la = int(rng.integers(3000, 8000))
        lb = int(rng.integers(600, 2500))
        a = rng.integers(0, 4, la).astype(np.uint8)
        start = int(rng.integers(0, la - lb))
        if t % 2 == 0:   # true stretch of A
            b = synth.mutate(rng, a[start:start + lb], 0.04, 0.03, 0.03)
        else:            # unrelated
            b = rng.integers(0, 4, lb).astype(np.uint8)
        pb = int(rng.integers(0, len(b) - 17))
        pa = start + pb if t % 2 == 0 else int(rng.integers(0, la - 17))
        pa = min(pa, la - 17)
        b[pb:pb + 17] = a[pa:pa + 17]
        if t % 4 >= 2:   # the short read as A: the range rides the edge i = m
            a, b, pa, pb = b, a, pb, pa
        a_l.append(a); b_l.append(b); pa_l.append(pa); pb_l.append(pb)
        x_l.append(int(rng.choice([100, 200, 400])))
    return synth.from_pairs(a_l, b_l, pa_l, pb_l, x_l, name=f"edge-riding[{seed}]")


@pytest.mark.parametrize("min_tier", [0, 3, 4, 5])
def test_bands_along_the_matrix_edge(ctx, xd, min_tier):
    """The wide tiers' assembly loop with ranges clipped to the matrix for
    long stretches (one read ends long before the other), from every
    register count; both extension directions."""
    bt = _edge_riding_pairs(min_tier)
    got = run(ctx, xd, bt, min_tier=min_tier)
    st = ctx.stats()
    assert st["jobs"][3:6].sum() > 0, st
    assert_same(got, oracle_of(bt), f"edge-riding from tier {min_tier}")


@pytest.mark.parametrize("impl", [0, 1])
def test_two_register_tier_cases(ctx, xd, impl):
    """The two-register tier's hand-scheduled loop and its C steps: bands of
    X = 60-100 that end inside the reads (a register empties), long X = 100
    requests (recentres, block boundaries, read ends), both directions."""
    from paper_2002_05200_amd import synth
    reqs = [r for r in (synth.make_request(i) for i in range(40)) if int(r.x[0]) == 100][:6]
    bt = synth.concat([_ending_pairs(0), _ending_pairs(1)] + reqs, name="two-register")
    ref = oracle_of(bt)
    assert_same(run(ctx, xd, bt, impl=impl), ref, f"impl {impl}")
    assert_same(run(ctx, xd, bt, impl=impl, min_tier=1), ref, f"impl {impl} from tier 1")
