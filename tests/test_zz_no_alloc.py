"""xdrop_extend_noalloc (no context, scratch in a fixed device array) against
xdrop_extend on the same inputs: every integer field bit-exact, on two calls
in a row whose second batch is smaller, under several launch options; the
oracle checks the first batch as well.  The array keeps the previous call's
contents, so the second call also shows that everything that must start at
zero is cleared.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
          "b_begin", "b_end", "left_cells", "right_cells", "status"]


def same(got, ref, label):
    for f in FIELDS:
        g, r = got[f].astype(np.int64), ref[f].astype(np.int64)
        bad = np.nonzero(g != r)[0]
        assert len(bad) == 0, (f"{label}: field {f} differs at pairs {bad[:10].tolist()} "
                               f"(noalloc {g[bad[:5]].tolist()} vs ref {r[bad[:5]].tolist()})")


def batches():
    from paper_2002_05200_amd import synth
    big = synth.concat([
        synth.random_cases(seed=4401, n=500, len_lo=17, len_hi=2500,
                           x_choices=(0, 1, 5, 10, 50, 100, 300, 1000), spurious_frac=0.4),
        synth.make_batch("uneven", n=120, start=11, stride=1601),
        synth.make_batch("batch10k", n=60, start=7, stride=1499),
    ], name="noalloc-big")
    small = synth.concat([
        synth.random_cases(seed=4402, n=150, len_lo=17, len_hi=900,
                           x_choices=(2, 10, 50, 100, 200)),
        synth.make_batch("plain1k", n=40, start=5),
    ], name="noalloc-small")
    return big, small


def test_noalloc_matches_xdrop_extend_on_two_calls():
    import torch
    from oracle import oracle
    from paper_2002_05200_amd import xdrop
    big, small = batches()
    assert small.n < big.n <= xdrop.NOALLOC_MAX_PAIRS
    ctx = xdrop.Context(0)
    try:
        option_sets = [None, dict(sched=1), dict(multi_wave=1, waves_per_cu=8),
                       dict(max_save_slots=3)]
        ref_big_oracle = oracle.batch(big)
        for kw in option_sets:
            opts = xdrop.make_opts(**kw) if kw is not None else None
            for bt in (big, small):
                print(f"[noalloc] {bt.name} n={bt.n} opts={kw}", flush=True)
                db = xdrop.DeviceBatch(bt, "cuda:0")
                ctx.extend_device(db, opts=opts)
                torch.cuda.synchronize()
                ref = db.results()
                db.d_out.fill_(0xAB)
                xdrop.extend_noalloc(db, device=0, opts=opts)
                torch.cuda.synchronize()
                got = db.results()
                same(got, ref, f"{bt.name} {kw}")
                if bt is big:
                    same(got, ref_big_oracle, f"{bt.name} {kw} vs oracle")
    finally:
        ctx.close()


def test_noalloc_band_wider_than_its_buffers_fails_that_pair_only():
    """A full-width band on 20 kb unrelated reads outgrows the fixed band
    buffers: that pair reports XD_ENOMEM, the others are exact."""
    import torch
    from oracle import oracle
    from paper_2002_05200_amd import synth, xdrop
    rng = np.random.default_rng(77)
    n = 20000
    a = rng.integers(0, 4, n, dtype=np.uint8)
    b = rng.integers(0, 4, n, dtype=np.uint8)
    b[100:117] = a[100:117]           # an exact 17-mer seed at (100, 100)
    wide = synth.from_pairs([a], [b], [100], [100], [1 << 20], name="wide")
    rest = synth.random_cases(seed=4403, n=64, len_lo=17, len_hi=600)
    bt = synth.concat([rest, wide, rest], name="noalloc-wide")
    db = xdrop.DeviceBatch(bt, "cuda:0")
    print(f"[noalloc] {bt.name} n={bt.n}", flush=True)
    xdrop.extend_noalloc(db, device=0)
    torch.cuda.synchronize()
    got = db.results()
    assert int(got["status"][64]) == xdrop.XD_ENOMEM
    ref = oracle.batch(rest)
    same(got[:64], ref, "before the wide pair")
    same(got[65:], ref, "after the wide pair")


def test_noalloc_rejects_what_it_cannot_hold():
    from paper_2002_05200_amd import synth, xdrop
    bt = synth.random_cases(seed=4404, n=4, len_lo=17, len_hi=100)
    db = xdrop.DeviceBatch(bt, "cuda:0")
    with pytest.raises(xdrop.XdropError) as e:
        xdrop.extend_noalloc(db, device=0, opts=xdrop.make_opts(profile=1))
    assert e.value.status == xdrop.XD_EINVAL
    L = xdrop.lib()
    st = L.xdrop_extend_noalloc(0, db.d_a.data_ptr(), len(db.a_words), db.d_b.data_ptr(),
                                len(db.b_words), db.d_pairs.data_ptr(),
                                xdrop.NOALLOC_MAX_PAIRS + 1, xdrop.Scores(1, -1, -1),
                                db.d_out.data_ptr(), None, None)
    assert st == xdrop.XD_EINVAL
    assert "XD_NOALLOC_MAX_PAIRS" in xdrop.last_error()
