"""GPU parity of xdrop_extend_matrix (4 x 4 substitution tables) against the
oracle's table form, bit-exact on every integer field.

Random tables (symmetric and not, narrow and wide value ranges), the
match/mismatch table (which must also equal xdrop_extend), DNA-style
transition/transversion tables, bands that outgrow the one-register window
and finish in the global-memory tier, degenerate pairs, and both launch
schedules."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ["score", "left_score", "right_score", "seed_score", "a_begin", "a_end",
          "b_begin", "b_end", "left_cells", "right_cells", "status"]


@pytest.fixture(scope="module")
def ctx():
    from paper_2002_05200_amd import xdrop
    c = xdrop.Context(0)
    yield c
    c.close()


def same(got, ref, label):
    for f in FIELDS:
        g, r = got[f].astype(np.int64), ref[f].astype(np.int64)
        bad = np.nonzero(g != r)[0]
        assert len(bad) == 0, (f"{label}: field {f} differs at pairs {bad[:8].tolist()} "
                               f"(gpu {g[bad[:4]].tolist()} oracle {r[bad[:4]].tolist()})")


def tables():
    r = np.random.default_rng(31)
    out = []
    for _ in range(3):
        t = r.integers(-3, 4, (4, 4))
        np.fill_diagonal(t, r.integers(1, 5, 4))
        out.append((f"random{len(out)}", t, -int(r.integers(1, 3))))
    sym = r.integers(-40, 10, (4, 4))
    sym = (sym + sym.T) // 2
    np.fill_diagonal(sym, r.integers(20, 60, 4))
    out.append(("symmetric wide", sym, -25))
    # transitions A<->G, C<->T score less badly than transversions
    ts = np.full((4, 4), -3)
    np.fill_diagonal(ts, 2)
    ts[0, 2] = ts[2, 0] = ts[1, 3] = ts[3, 1] = -1
    out.append(("transition/transversion", ts, -2))
    asym = r.integers(-5, 3, (4, 4))
    np.fill_diagonal(asym, [1, 2, 3, 4])
    out.append(("asymmetric", asym, -1))
    return out


@pytest.mark.parametrize("case", range(6))
def test_random_and_dna_tables(ctx, case):
    from oracle import oracle
    from paper_2002_05200_amd import synth
    name, t, gap = tables()[case]
    bt = synth.random_cases(seed=800 + case, n=257, len_lo=17, len_hi=1200,
                            x_choices=(0, 1, 3, 10, 30, 60, 150))
    print(f"[matrix] {name} gap {gap} n={bt.n}", flush=True)
    ref = oracle.batch_matrix(bt, t, gap)
    same(ctx.extend_matrix(bt, t, gap), ref, name)


def test_linear_table_equals_xdrop_extend(ctx):
    from oracle import oracle
    from paper_2002_05200_amd import synth, xdrop
    bt = synth.concat([synth.random_cases(seed=850, n=200, len_lo=17, len_hi=900,
                                          x_choices=(0, 2, 10, 40)),
                       synth.make_batch("batch10k", n=12, start=9, stride=7001)], name="linear")
    t = np.full((4, 4), -1)
    np.fill_diagonal(t, 1)
    got = ctx.extend_matrix(bt, t, -1)
    same(got, ctx.extend(bt), "table vs xdrop_extend")
    same(got, oracle.batch(bt), "table vs oracle")
    same(ctx.extend_matrix(bt, t, -1, opts=xdrop.make_opts(sched=xdrop.SCHED_PLAIN)), got, "plain")


def test_wide_bands_finish_in_global_memory(ctx):
    """Unrelated reads at large X: bands outgrow the 62-slot window, restart in
    the global-memory tier, and still match the oracle."""
    from oracle import oracle
    from paper_2002_05200_amd import synth
    t = np.array([[3, -2, -1, -2], [-2, 3, -2, -1], [-1, -2, 3, -2], [-2, -1, -2, 3]])
    bt = synth.random_cases(seed=860, n=60, len_lo=300, len_hi=2500,
                            x_choices=(80, 200, 600), spurious_frac=0.8)
    got = ctx.extend_matrix(bt, t, -2)
    st = ctx.stats()
    assert st["jobs"][6] > 0 and st["restarted"][0] > 0, st
    same(got, oracle.batch_matrix(bt, t, -2), "wide bands")


def test_degenerate_pairs_and_errors(ctx):
    from oracle import oracle
    from paper_2002_05200_amd import synth, xdrop
    r = np.random.default_rng(870)
    a_l, b_l, pa, pb, xs = [], [], [], [], []
    for _ in range(120):
        L = int(r.integers(0, 30))
        a = r.integers(0, 4, L).astype(np.uint8)
        b = a.copy() if r.random() < 0.5 else r.integers(0, 4, int(r.integers(0, 30))).astype(np.uint8)
        p = int(r.integers(0, min(len(a), len(b)) + 1))
        a_l.append(a); b_l.append(b); pa.append(p); pb.append(p); xs.append(int(r.integers(0, 6)))
    bt = synth.from_pairs(a_l, b_l, pa, pb, xs, k=0, name="degenerate")
    t = r.integers(-2, 3, (4, 4))
    same(ctx.extend_matrix(bt, t, -1), oracle.batch_matrix(bt, t, -1), "degenerate")
    db = xdrop.DeviceBatch(bt, "cuda:0")
    with pytest.raises(xdrop.XdropError):
        ctx.extend_device_matrix(db, np.full((4, 4), 1 << 21), -1)
    with pytest.raises(xdrop.XdropError):
        ctx.extend_device_matrix(db, t, 1)
    with pytest.raises(xdrop.XdropError):
        ctx.extend_device_matrix(db, t, -1, opts=xdrop.make_opts(graph=1))
