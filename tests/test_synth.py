"""The seeded generator: determinism, shapes and the planted exact seeds."""
import numpy as np

from paper_2002_05200_amd import synth


def test_pairs_are_reproducible_and_independent_of_batching():
    a = synth.make_batch("batch10k", n=40, start=0)
    b = synth.make_batch("batch10k", n=20, start=20)
    for p in range(20):
        x1, y1 = a.pair(20 + p)
        x2, y2 = b.pair(p)
        assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
        assert a.a_seed[20 + p] == b.a_seed[p] and a.b_seed[20 + p] == b.b_seed[p]


def test_seeds_are_exact_kmers():
    for w in ("plain1k", "batch10k", "uneven"):
        bt = synth.make_batch(w, n=50)
        for p in range(bt.n):
            a, b = bt.pair(p)
            pa, pb = int(bt.a_seed[p]), int(bt.b_seed[p])
            assert 0 <= pa <= len(a) - bt.k and 0 <= pb <= len(b) - bt.k
            assert np.array_equal(a[pa:pa + bt.k], b[pb:pb + bt.k])


def test_workload_shapes():
    bt = synth.make_batch("plain1k", n=100)
    assert (bt.a_len == 1000).all() and (bt.x == 10).all()
    assert ((bt.a_seed >= 450) & (bt.a_seed <= 533)).all()
    bt = synth.make_batch("batch10k", n=400)
    assert bt.a_len.min() >= 1000 and bt.a_len.max() <= 40000
    assert 7000 < np.median(bt.a_len) < 14000
    bt = synth.make_batch("uneven", n=300)
    assert bt.a_len.min() >= 500 and bt.a_len.max() <= 100000


def test_error_channel_rates():
    rng = synth.pair_rng(77, 0)
    t = synth.random_bases(rng, 200000)
    out = synth.mutate(rng, t, 0.05, 0.05, 0.05)
    # deletions remove 5%, insertions add 5%: length within 1% of the template
    assert abs(len(out) - len(t)) < 0.01 * len(t)
    out0 = synth.mutate(rng, t, 0.0, 0.0, 0.0)
    assert np.array_equal(out0, t)
    subs = synth.mutate(rng, t, 0.2, 0.0, 0.0)
    frac = (subs != t).mean()
    assert 0.19 < frac < 0.21


def test_serving_requests():
    for r in range(5):
        bt = synth.make_request(r)
        assert 1 <= bt.n <= 64
        assert len(set(bt.x.tolist())) == 1 and int(bt.x[0]) in synth.SERVING_X
    t = synth.poisson_arrivals(1000, 50.0)
    assert np.all(np.diff(t) > 0) and 15 < t[-1] < 25


def test_encode_decode_roundtrip():
    s = "ACGTTGCA"
    assert synth.decode(synth.encode(s)) == s.encode()


def _worker_pid(_):
    import os
    return os.getpid()


def test_pool_map_matches_a_serial_map_and_lets_workers_exit():
    # the same results, in order, as a plain map
    assert synth.pool_map(abs, [-3, 4, -5, 6, -7], 2) == [3, 4, 5, 6, 7]
    # the workers are joined before it returns: none of them is still alive
    import os
    pids = set(synth.pool_map(_worker_pid, range(8), 2))
    assert os.getpid() not in pids
    for pid in pids:
        try:
            os.kill(pid, 0)
            alive = True
        except ProcessLookupError:
            alive = False
        assert not alive
