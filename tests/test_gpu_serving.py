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
    """A slot share that holds only a few requests: the queue drains batch
    by batch and every result still equals the unconstrained run."""
    ref_srv = xd.Server(slots=2, max_batch_pairs=256)
    try:
        ref = run_all(ref_srv, xd, requests[:12])
    finally:
        ref_srv.close()
    words = [(len(xd.pack_codes(bt.a)), len(xd.pack_codes(bt.b))) for bt in requests[:12]]
    cap_words = max(max(w) for w in words) + 64           # one slot: the largest request + a little
    share = cap_words * 8 + 256 * (40 + 56)
    srv = xd.Server(slots=2, max_batch_pairs=256, mem_budget=2 * share)
    try:
        got = run_all(srv, xd, requests[:12])
        for r in range(12):
            assert same(got[r], ref[r]), f"request {r}"
        # admission by memory: no batch held more read words than a slot has
        least = -(-sum(a for a, _ in words) // cap_words)
        assert srv.stats()["batches"] >= max(least, 2), (srv.stats(), least)
    finally:
        srv.close()


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
