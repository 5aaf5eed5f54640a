"""Serving loop on the GPU: continuous batching gives every request the same
results alone and in a mix (tolerance 0), equal to the CPU oracle, with and
without graph replay, under tight admission memory."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
          "b_begin", "b_end", "left_cells", "right_cells", "status"]


def same(a, b):
    return all(np.array_equal(a[f], b[f]) for f in FIELDS)


@pytest.fixture(scope="module")
def xd():
    from paper_2002_05200_amd import xdrop
    return xdrop


@pytest.fixture(scope="module")
def requests():
    from paper_2002_05200_amd import synth
    return [synth.make_request(r) for r in range(40)]


def oracle_of(bt):
    from oracle import oracle
    return oracle.batch(bt)


def run_all(srv, xd, reqs):
    packed = [xd.PackedRequest(bt) for bt in reqs]
    tickets = [srv.submit(p) for p in packed]
    out = []
    for t, p in zip(tickets, packed):
        got = srv.poll(t, p.n, wait_ms=60000)
        assert got is not None, "request not done within 60 s"
        out.append(got[0])
    return out


@pytest.mark.parametrize("graph", [0, 1])
def test_alone_and_in_a_mix_agree_with_the_oracle(xd, requests, graph):
    print(f"serving graph={graph}", flush=True)
    srv = xd.Server(slots=4, max_batch_pairs=512, graph=graph, mem_budget=256 << 20)
    try:
        probe = [0, 7, 23]
        alone = {r: run_all(srv, xd, [requests[r]])[0] for r in probe}
        mix = run_all(srv, xd, requests)               # all 40 submitted back to back
        for r in probe:
            assert same(alone[r], mix[r]), f"request {r} differs alone vs in the mix"
        for r in probe + [39]:
            ref = oracle_of(requests[r])
            assert same(mix[r], ref), f"request {r} differs from the oracle"
        st = srv.stats()
        assert st["requests"] == len(requests) + len(probe)
        assert st["pairs"] == sum(bt.n for bt in requests) + sum(requests[r].n for r in probe)
        assert st["max_inflight"] >= 2, st                  # batches overlapped on the device
    finally:
        srv.close()


def test_tight_admission_memory_still_completes_everything(xd, requests):
    """A memory budget whose slot arenas hold only a few requests: the queue
    drains batch by batch, every result still equals the unconstrained run,
    and the slots' device memory stays inside the budget."""
    ref_srv = xd.Server(slots=2, max_batch_pairs=256)
    try:
        ref = run_all(ref_srv, xd, requests[:12])
    finally:
        ref_srv.close()
    words = [(len(xd.pack_codes(bt.a)), len(xd.pack_codes(bt.b))) for bt in requests[:12]]
    budget = 2 * (7 << 19)                                # two slots of 3.5 MiB
    srv = xd.Server(slots=2, max_batch_pairs=256, mem_budget=budget)
    try:
        st0 = srv.stats()
        assert 0 < st0["device_bytes"] <= budget, st0
        cap_words = st0["arena_words"]
        assert max(max(w) for w in words) <= cap_words < sum(a for a, _ in words), (cap_words, words)
        got = run_all(srv, xd, requests[:12])
        for r in range(12):
            assert same(got[r], ref[r]), f"request {r}"
        # admission by memory: no batch held more read words than a slot has
        least = -(-sum(a for a, _ in words) // cap_words)
        assert srv.stats()["batches"] >= max(least, 2), (srv.stats(), least)
    finally:
        srv.close()


def test_device_memory_stays_inside_the_budget(xd):
    for slots, budget in [(1, 64 << 20), (4, 1 << 30), (16, 2 << 30)]:
        srv = xd.Server(slots=slots, max_batch_pairs=2048, mem_budget=budget)
        try:
            st = srv.stats()
            assert 0 < st["device_bytes"] <= budget, (slots, budget, st)
        finally:
            srv.close()
    with pytest.raises(xd.XdropError) as e:        # too small for one slot's context
        xd.Server(slots=4, max_batch_pairs=2048, mem_budget=4 << 20)
    assert e.value.status == xd.XD_EINVAL


def test_cancel_and_destroy(xd, requests):
    """Requests still queued can be canceled (their polls say so); requests
    on the device finish; destroying the server cancels what is queued and
    wakes every poll waiting inside it."""
    import threading
    srv = xd.Server(slots=1, max_batch_pairs=64, mem_budget=64 << 20)
    packed = [xd.PackedRequest(bt) for bt in requests[:10]]
    tickets = [srv.submit(p) for p in packed]
    outcome = {}
    for t in tickets[::-1]:                        # newest first: most are still queued
        outcome[t] = srv.cancel(t)
    assert xd.XD_OK in outcome.values()
    for t, p in zip(tickets, packed):
        if outcome[t] == xd.XD_OK:
            with pytest.raises(xd.XdropError) as e:
                srv.poll(t, p.n, wait_ms=-1)
            assert e.value.status == xd.XD_ECANCELED
        else:
            assert outcome[t] == xd.XD_EBUSY
            assert srv.poll(t, p.n, wait_ms=60000) is not None
    with pytest.raises(xd.XdropError):
        srv.cancel(tickets[0])                     # released by its poll: unknown now
    assert srv.stats()["canceled"] == sum(v == xd.XD_OK for v in outcome.values())
    # destroy with requests queued and polls waiting on them
    tickets = [srv.submit(p) for p in packed]
    results = {}

    def wait(t, n):
        try:
            results[t] = srv.poll(t, n, wait_ms=-1)
        except xd.XdropError as e:
            results[t] = e.status

    threads = [threading.Thread(target=wait, args=(t, p.n)) for t, p in zip(tickets, packed)]
    for th in threads:
        th.start()
    import time
    t0 = time.time()                               # every poll is inside the server or done
    while srv.stats()["waiting_polls"] + len(results) < len(threads):
        assert time.time() - t0 < 60
        time.sleep(0.001)
    srv.close()
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive()
    assert len(results) == len(tickets)
    assert all(v == xd.XD_ECANCELED or (isinstance(v, tuple)) for v in results.values())


def test_watchdog_fails_slow_batches_and_the_server_goes_on(xd, requests):
    """A watchdog shorter than most batches: their requests fail with
    XD_ETIMEDOUT as soon as it fires, while their kernels still run to the end
    (nothing on the GPU is interrupted); requests that finish in time are
    exact; the slots are reused and the server shuts down cleanly."""
    srv = xd.Server(slots=2, max_batch_pairs=256, mem_budget=256 << 20, watchdog_ms=1)
    try:
        packed = [xd.PackedRequest(bt) for bt in requests[:10]]
        outcome = []
        for rnd in range(2):                      # a second round reuses the drained slots
            tickets = [srv.submit(p) for p in packed]
            for r, (t, p) in enumerate(zip(tickets, packed)):
                try:
                    got = srv.poll(t, p.n, wait_ms=60000)
                    assert got is not None
                    assert same(got[0], oracle_of(requests[r])), f"request {r}"
                    outcome.append("ok")
                except xd.XdropError as e:
                    assert e.status == xd.XD_ETIMEDOUT, e
                    outcome.append("timed out")
        print(f"[serving] watchdog outcomes {outcome}", flush=True)
        assert "timed out" in outcome
        assert srv.stats()["timed_out"] == outcome.count("timed out")
    finally:
        srv.close()
    with pytest.raises(xd.XdropError):
        xd.Server(slots=1, watchdog_ms=-1)


def test_oversized_request_is_rejected(xd, requests):
    srv = xd.Server(slots=1, max_batch_pairs=4, mem_budget=8 << 20)
    try:
        big = next(bt for bt in requests if bt.n > 4)
        with pytest.raises(xd.XdropError) as e:
            srv.submit(xd.PackedRequest(big))
        assert e.value.status == xd.XD_EINVAL
        assert "larger than a slot" in xd.last_error()
    finally:
        srv.close()
