"""Lazy deletion on the GPU (GPMA_FLAG_LAZY_DELETE) against the oracle's lazy
mode, slot for slot: marked entries (bit 63) in the same places, the same
leaf counts (occupied slots), row offsets, degrees and live edge count; the
analytics over the live edges; fused sequences equal to plain ones; the
mirror marked alike.

The oracle's lazy mode is pinned on the CPU (tests/test_oracle.py): marks
only the deleted entries, keeps the live set equal to the eager mode's, and
recycles marked slots on the next merge."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

PR_RTOL = 1e-6
TOMB = np.uint64(1 << 63)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(keys) -> torch.Tensor:
    if isinstance(keys, torch.Tensor):
        return keys.to("cuda")
    return torch.from_numpy(np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).view(np.int64)).cuda()


def npu64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def transpose(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, dtype=np.uint64)
    return (k << np.uint64(32)) | (k >> np.uint64(32))


def make(V, init, lf, **kw):
    from paper_1709_05061_amd import GPMA
    init = np.asarray(init, dtype=np.uint64)
    g = GPMA(V, dev(init), leaf_size=lf, lazy_delete=True, **kw)
    ref = O.OraclePMA(V, init, lf, lazy=True)
    return g, ref


def check_state(g, ref, V):
    slots = npu64(g.slots())
    want = ref.slots()
    assert g.capacity == ref.capacity, (g.capacity, ref.capacity)
    if not np.array_equal(slots, want):
        bad = np.nonzero(slots != want)[0]
        raise AssertionError("slots differ at %d positions, first %s: gpu %x oracle %x"
                             % (bad.size, bad[:5], slots[bad[0]], want[bad[0]]))
    lf = g.leaf_size
    assert np.array_equal(g.leaf_counts().cpu().numpy().astype(np.int64), O.leaf_counts(want, lf))
    assert np.array_equal(npu64(g.pivots()), O.leaf_pivots(want, lf))
    assert np.array_equal(g.row_offsets().cpu().numpy().astype(np.int64), O.row_offsets(want, V))
    edges = O.edge_keys(want)
    assert np.array_equal(g.degrees().cpu().numpy().astype(np.int64), O.out_degrees(edges, V))
    assert g.num_edges == edges.size
    assert np.array_equal(npu64(g.keys()), edges)
    return edges


def marked(slots: np.ndarray) -> int:
    return int(np.count_nonzero((slots != O.EMPTY) & ((slots & TOMB) != 0)))


def run_stream(g, ref, V, batches, mref=None, pr_every=0):
    from test_gpu_pma import check_merge_log
    for t, (op, keys) in enumerate(batches):
        cap0 = ref.capacity
        st = getattr(g, op)(dev(keys), stats=True)
        getattr(ref, op)(keys)
        check_merge_log(st, ref, g.leaf_size, cap0)
        if mref is not None:
            getattr(mref, op)(transpose(keys))
        assert st.applied == ref.last_applied(), (t, op, st.applied, ref.last_applied())
        if op == "delete":
            assert st.top_level <= 0 and not st.resized, (t, st)
        edges = check_state(g, ref, V)
        if mref is not None:
            m = g.mirror()
            assert np.array_equal(npu64(m.slots()), mref.slots()), t
            assert np.array_equal(m.row_offsets().cpu().numpy().astype(np.int64),
                                  O.row_offsets(mref.slots(), V))
        if pr_every and t % pr_every == 0:
            x = g.pagerank(iters=10).cpu().numpy()
            want = O.pagerank(V, edges, iters=10)
            assert np.max(np.abs(x - want) / want) < PR_RTOL, t


@pytest.mark.parametrize("mirror", [False, True])
def test_lazy_sliding_window_er(mirror):
    """ER sliding window (2^12 vertices, 2^15 edges, slides of 2^9): deletes
    mark, inserts merge and recycle marked slots; the mirror is marked alike."""
    V, W, b, S = 1 << 12, 1 << 15, 1 << 9, 8
    st = synth.er_stream(V, W, b, S, seed=31)
    init = npu64(st.initial())
    g, ref = make(V, init, 32, mirror=mirror)
    mref = O.OraclePMA(V, transpose(init), 32, lazy=True) if mirror else None
    batches = []
    for t in range(S):
        d, i = st.slide(t, b)
        batches += [("delete", npu64(d)), ("insert", npu64(i))]
    say("lazy sliding window, mirror", mirror)
    run_stream(g, ref, V, batches, mref=mref, pr_every=5)
    assert marked(npu64(g.slots())) > 0
    g.close()


@pytest.mark.parametrize("tier_lds", [0, 1])
def test_lazy_growth_marks_and_recycling(tier_lds):
    """A small graph grown past several doublings (the root rebuild drops
    marks), most of it deleted (marks only: capacity stays), then the
    deleted keys inserted again (merges recycle marked slots and climb
    levels); with tier_lds=1 every level above the leaves runs through the
    device tier (live-count offsets, ballot gather)."""
    V, lf = 64, 16
    rng = np.random.default_rng(7)
    allk = np.array([(u << 32) | v for u in range(V) for v in range(V)], dtype=np.uint64)
    rng.shuffle(allk)
    g, ref = make(V, allk[:40], lf, lds_tier=tier_lds)
    batches = []
    pos = 40
    for sz in [3, 17, 200, 500, 999]:
        kk = allk[pos:pos + sz]
        pos += sz
        batches.append(("insert", np.concatenate([kk, kk[:2], allk[:5]])))
    live = allk[:pos]
    gone = []
    for sz in [700, 900, 150, 1]:
        idx = rng.choice(live.size, min(sz, live.size), replace=False)
        kk = live[idx]
        live = np.delete(live, idx)
        gone.append(kk)
        # repeats, and an already marked key: no-ops
        batches.append(("delete", np.concatenate([kk, kk[:3], gone[0][:2] if len(gone) > 1 else kk[:0]])))
    back = np.concatenate(gone)
    rng.shuffle(back)
    for a in range(0, back.size, 400):
        batches.append(("insert", back[a:a + 400]))
    batches.append(("insert", allk[pos:pos + 1200]))   # new keys: the root doubles over marks
    say("lazy growth", tier_lds, len(batches))
    run_stream(g, ref, V, batches, pr_every=4)
    g.close()


@pytest.mark.parametrize("lf", [16, 64, 256, 512])
def test_lazy_leaf_sizes(lf):
    V = 2000
    st = synth.er_stream(V, 30000, 3000, 3, seed=40 + lf)
    g, ref = make(V, npu64(st.initial()), lf)
    batches = []
    for t in range(3):
        d, i = st.slide(t, 3000)
        batches += [("delete", npu64(d)), ("insert", npu64(i))]
    batches.append(("insert", npu64(synth.random_batch(V, 5000, 99))))
    run_stream(g, ref, V, batches)
    g.close()


def test_lazy_rmat_learned_locator():
    """R-MAT scale 13: marked pivots must not change the learned locator's
    leaves (the model and its bracket checks read masked pivots)."""
    st = synth.rmat_stream(13, 16, seed=12)
    V = st.V
    init = npu64(st.initial())
    g, ref = make(V, init, 32, learned=True, mirror=True)
    mref = O.OraclePMA(V, transpose(init), 32, lazy=True)
    t0 = 0
    batches = []
    for lb in (8, 10, 12, 12):
        b = 1 << lb
        d, i = st.order[t0:t0 + b], st.order[st.window + t0: st.window + t0 + b]
        t0 += b
        batches += [("delete", npu64(d)), ("insert", npu64(i))]
    run_stream(g, ref, V, batches, mref=mref)
    info = g.locator_info()
    assert info["lookups"] > 0
    g.close()


@pytest.mark.parametrize("mirror,direct,levels", [(False, False, 1), (True, True, 0), (True, False, 2)])
def test_lazy_fused_equals_plain(mirror, direct, levels):
    """Fused sequences with lazy deletes equal the plain path and the oracle
    (a lazy delete batch is select, locate, mark: it never stops the
    sequence)."""
    from paper_1709_05061_amd import GPMA
    V, lf = 512, 16
    rng = np.random.default_rng(17)
    init = np.unique(npu64(synth.random_batch(V, 6000, 3)))
    live = set(int(x) for x in init)
    ops, bs = [], []
    for t in range(30):
        size = int(2 ** rng.uniform(3, 11))
        if rng.random() < 0.5 or len(live) < 2 * size:
            keys = np.array([(int(a) << 32) | int(b) for a, b in
                             zip(rng.integers(0, V, size), rng.integers(0, V, size))], np.uint64)
            op = 0
            live |= set(int(x) for x in keys)
        else:
            pool = np.array(sorted(live), np.uint64)
            keys = pool[rng.choice(pool.size, size, replace=False)]
            op = 1
            live -= set(int(x) for x in keys)
        ops.append(op)
        bs.append(np.concatenate([keys, keys[: max(1, keys.size // 10)]]))
    plain = GPMA(V, dev(init), leaf_size=lf, mirror=mirror, lazy_delete=True)
    fused = GPMA(V, dev(init), leaf_size=lf, mirror=mirror, lazy_delete=True, fused_direct=direct,
                 fused_levels=levels)
    ref = O.OraclePMA(V, init, lf, lazy=True)
    for lo, hi in ((0, 7), (7, 8), (8, 30)):
        say("lazy fused", lo, hi, mirror, direct, levels)
        for i in range(lo, hi):
            (plain.delete if ops[i] else plain.insert)(dev(bs[i]))
            (ref.delete if ops[i] else ref.insert)(bs[i])
        s = fused.apply_batches(ops[lo:hi], [dev(b) for b in bs[lo:hi]])
        assert np.array_equal(npu64(fused.slots()), npu64(plain.slots())), (lo, hi)
        assert np.array_equal(npu64(fused.slots()), ref.slots())
        assert fused.num_edges == plain.num_edges
        assert np.array_equal(fused.degrees().cpu().numpy(), plain.degrees().cpu().numpy())
        if mirror:
            assert np.array_equal(npu64(fused.mirror().slots()), npu64(plain.mirror().slots()))
    assert marked(npu64(fused.slots())) > 0
    plain.close()
    fused.close()


@pytest.mark.parametrize("mode", ["binned", "binned_gather", "pull", "push"])
def test_lazy_analytics_skip_marks(mode):
    """PageRank (every SpMV form), BFS (top-down and, over the mirror,
    bottom-up) and CC (label propagation and the sampling path) over an
    array with many marked entries equal the oracle on the live edges."""
    u = npu64(synth.rmat_unique(13, 16 << 13, seed=8))
    V = 1 << 13
    g, ref = make(V, u, 32, mirror=mode == "pull", spmv=mode)
    rng = np.random.default_rng(5)
    d = u[rng.choice(u.size, u.size // 2, replace=False)]
    g.delete(dev(d))
    ref.delete(d)
    e = check_state(g, ref, V)
    assert marked(npu64(g.slots())) == d.size
    x = g.pagerank(iters=10).cpu().numpy()
    want = O.pagerank(V, e, iters=10)
    assert np.max(np.abs(x - want) / want) < PR_RTOL
    for src in (0, 1, V // 2):
        assert np.array_equal(g.bfs(src).cpu().numpy(), O.bfs(V, e, src)), src
    assert np.array_equal(g.cc().cpu().numpy().astype(np.uint32), O.cc(V, e))
    g.close()


def test_lazy_delete_everything_then_reinsert():
    """Every edge marked: the analytics see an edgeless graph; inserting the
    keys again merges them back over their marks."""
    V = 300
    init = np.unique(npu64(synth.random_batch(V, 3000, 2)))
    g, ref = make(V, init, 16, mirror=True)
    mref = O.OraclePMA(V, transpose(init), 16, lazy=True)
    run_stream(g, ref, V, [("delete", init)], mref=mref)
    assert g.num_edges == 0 and marked(npu64(g.slots())) == init.size
    np.testing.assert_allclose(g.pagerank(iters=3).cpu().numpy(), 1.0 / V, rtol=1e-6)
    assert list(g.bfs(7).cpu().numpy()) == [-1] * 7 + [0] + [-1] * (V - 8)
    assert list(g.cc().cpu().numpy()) == list(range(V))
    run_stream(g, ref, V, [("delete", init[:10]), ("insert", init[::2]), ("insert", init)], mref=mref)
    g.close()
