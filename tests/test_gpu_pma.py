"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Layout parity is slot for slot: the GPU's raw slot array, leaf counts, CSR
row offsets and degrees must equal what the sequential oracle produces from
the same seeded inputs.  BFS and CC must match exactly; PageRank within
1e-6 max relative error (each of the 10 fp32 roundings adds at most 2^-24
relative error to positive terms, so 10 steps stay below 6e-7).
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

PR_RTOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(keys) -> torch.Tensor:
    if isinstance(keys, torch.Tensor):
        return keys.to("cuda")
    return torch.from_numpy(np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).view(np.int64)).cuda()


def npu64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def check_state(g, ref, V):
    slots = npu64(g.slots())
    want = ref.slots()
    assert g.capacity == ref.capacity
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
    return edges


def make(V, init, lf, mirror=False, gpu_kw=None, **kw):
    from paper_1709_05061_amd import GPMA
    init_np = np.asarray(init.numpy() if isinstance(init, torch.Tensor) else init).view(np.uint64) \
        if len(init) else np.zeros(0, np.uint64)
    g = GPMA(V, dev(init_np), leaf_size=lf, mirror=mirror, **kw, **(gpu_kw or {}))
    ref = O.OraclePMA(V, init_np, lf, **kw)
    return g, ref


@pytest.mark.parametrize("V,n,lf,seed", [(3, 0, 16, 0), (100, 0, 16, 1), (1000, 5000, 16, 2),
                                         (1 << 14, 1 << 17, 32, 3), (5000, 40000, 64, 4),
                                         (777, 3000, 128, 5)])
def test_create_matches_oracle(V, n, lf, seed):
    say("create", V, n, lf, seed)
    init = synth.random_batch(V, n, seed)
    g, ref = make(V, init, lf)
    check_state(g, ref, V)
    g.close()


def test_create_csr_example_and_auto_leaf():
    from paper_1709_05061_amd import GPMA
    keys = [(0 << 32) | 0, (0 << 32) | 2, (1 << 32) | 2, (2 << 32) | 0, (2 << 32) | 1, (2 << 32) | 2]
    g = GPMA(3, dev(keys))
    assert g.leaf_size == 16
    ref = O.OraclePMA(3, np.array(keys, np.uint64), 16)
    check_state(g, ref, 3)
    ro = g.row_offsets().cpu().numpy()
    assert ro[0] == 0 and list(npu64(g.keys())) == sorted(keys)
    g.close()


def check_merge_log(st, ref, lf, cap_before):
    """The batch's merges, level by level, equal the oracle's merge log
    (Example 3 of Section 5.2 narrates such rounds): as many segments merged
    at every height, the root counted at the old height whether it took the
    batch in place or was rebuilt at a new capacity, and the same sum of
    rewritten segment capacities."""
    H = int(np.log2(cap_before // lf))
    want = {}
    rew = 0
    for lvl, seg in ref.merge_log():
        h = H if lvl < 0 else lvl
        want[h] = want.get(h, 0) + 1
        rew += seg if lvl < 0 else lf << lvl
    got = {h: c for h, c in enumerate(st.segments_merged) if c}
    assert got == want, (got, want)
    assert st.slots_rewritten == rew, (st.slots_rewritten, rew)
    assert st.top_level == (max(want) if want else -1)


def run_stream(g, ref, V, batches, pr_every=0, check_every=1):
    """batches: list of (op, numpy uint64 keys)."""
    x = None
    for t, (op, keys) in enumerate(batches):
        cap0 = ref.capacity
        st = getattr(g, op)(dev(keys), stats=True)
        getattr(ref, op)(keys)
        assert st.applied == ref.last_applied(), (t, op, st, ref.last_applied())
        assert st.noops == ref.last_noops(), (t, op, st.noops, ref.last_noops())
        check_merge_log(st, ref, g.leaf_size, cap0)
        if t % check_every == 0 or t == len(batches) - 1:
            edges = check_state(g, ref, V)
            if pr_every and t % pr_every == 0:
                x = g.pagerank(init=x, iters=10)
                want = O.pagerank(V, edges, x0=None if t == 0 else xin, iters=10)
                rel = np.max(np.abs(x.cpu().numpy() - want) / want)
                assert rel < PR_RTOL, (t, rel)
            xin = None if x is None else x.cpu().numpy().astype(np.float64)


def test_sliding_window_er_2e14():
    """Uniform random graph, 2^14 vertices, 2^17 initial edges, 32 slides of
    2^10 deletes (oldest) + 2^10 inserts; PageRank after every slide."""
    V, W, b, S = 1 << 14, 1 << 17, 1 << 10, 32
    st = synth.er_stream(V, W, b, S, seed=1)
    g, ref = make(V, st.initial(), 32)
    check_state(g, ref, V)
    x = None
    for t in range(S):
        say("slide", t)
        d, i = st.slide(t, b)
        sd = g.delete(dev(d), stats=True)
        ref.delete(npu64(d))
        assert sd.applied == b and ref.last_applied() == b
        si = g.insert(dev(i), stats=True)
        ref.insert(npu64(i))
        assert si.applied == b
        edges = check_state(g, ref, V)
        xin = None if x is None else x.cpu().numpy().astype(np.float64)
        x = g.pagerank(init=x, iters=10, out=None)
        want = O.pagerank(V, edges, x0=xin, iters=10)
        rel = np.max(np.abs(x.cpu().numpy() - want) / want)
        assert rel < PR_RTOL, (t, rel)
    g.close()


@pytest.mark.parametrize("tier_lds", [0, 1])
def test_growth_and_shrink_climbs_levels(tier_lds):
    """Small graph grown well past several doublings and shrunk back: every
    level of the tree and the root resize are exercised; with the workgroup
    tier capped at 1 byte of LDS the levels above the leaves run through the
    device tier."""
    V, lf = 64, 16
    rng = np.random.default_rng(3)
    allk = np.array([(u << 32) | v for u in range(V) for v in range(V)], dtype=np.uint64)
    rng.shuffle(allk)
    g, ref = make(V, allk[:40], lf, gpu_kw=dict(lds_tier=tier_lds))
    batches = []
    pos = 40
    for sz in [1, 3, 17, 64, 200, 333, 500, 800, 999, 1]:
        kk = allk[pos:pos + sz]
        pos += sz
        extra = allk[:5]                      # present keys: no-ops
        batches.append(("insert", np.concatenate([kk, kk[:2], extra])))
    live = allk[:pos]
    for sz in [700, 900, 1000, 500, 300, 100, 10, 3]:
        idx = rng.choice(live.size, min(sz, live.size), replace=False)
        kk = live[idx]
        live = np.delete(live, idx)
        batches.append(("delete", np.concatenate([kk, kk[:3]])))
    say("growth/shrink", tier_lds, len(batches))
    run_stream(g, ref, V, batches, pr_every=3)
    g.close()


def test_sorted_stream_is_adversarial_but_exact():
    """Sorted arrivals all land at the right end of the array (the worst case
    for segment cascades)."""
    V, lf = 256, 16
    allk = np.array([(u << 32) | v for u in range(V) for v in range(0, V, 3)], dtype=np.uint64)
    g, ref = make(V, allk[:500], lf)
    batches = [("insert", allk[p:p + 400]) for p in range(500, allk.size, 400)]
    batches += [("delete", allk[p:p + 700]) for p in range(0, allk.size, 700)]
    run_stream(g, ref, V, batches)
    g.close()


@pytest.mark.parametrize("lf", [16, 32, 64, 128, 256, 512])
def test_leaf_sizes(lf):
    V = 2000
    st = synth.er_stream(V, 30000, 3000, 4, seed=lf)
    g, ref = make(V, st.initial(), lf)
    batches = []
    for t in range(4):
        d, i = st.slide(t, 3000)
        batches += [("delete", npu64(d)), ("insert", npu64(i))]
    batches.append(("insert", npu64(synth.random_batch(V, 5000, 99))))
    run_stream(g, ref, V, batches)
    g.close()


def test_rmat_stream_batch_sizes():
    """R-MAT (a=.57, b=c=.19) scale 14, edge factor 16; slides of 2^6..2^12."""
    st = synth.rmat_stream(14, 16, seed=2)
    V = st.V
    g, ref = make(V, st.initial(), 32)
    check_state(g, ref, V)
    t0 = 0
    for lb in (6, 8, 10, 12):
        b = 1 << lb
        for _ in range(2):
            d, i = st.order[t0:t0 + b], st.order[st.window + t0: st.window + t0 + b]
            t0 += b
            say("rmat slide b=", b)
            run_stream(g, ref, V, [("delete", npu64(d)), ("insert", npu64(i))])
    g.close()


def test_invalid_batch_changes_nothing():
    from paper_1709_05061_amd import GpmaError
    V = 50
    g, ref = make(V, synth.random_batch(V, 300, 1), 16)
    before = npu64(g.slots())
    for bad in ((V << 32) | 1, (1 << 32) | V, (3 << 32) | 0xFFFFFFFF):
        for op in ("insert", "delete"):
            with pytest.raises(GpmaError) as ei:
                getattr(g, op)(dev([(1 << 32) | 2, bad]))
            assert ei.value.code == -1
    assert np.array_equal(npu64(g.slots()), before)
    check_state(g, ref, V)
    g.close()


def test_empty_repeated_and_noop_batches():
    V = 40
    init = npu64(synth.random_batch(V, 200, 4))
    g, ref = make(V, init, 16)
    st = g.insert(dev(np.zeros(0, np.uint64)), stats=True)
    assert st.applied == 0
    present = np.unique(init)[:30]
    st = g.insert(dev(np.concatenate([present, present])), stats=True)
    assert st.applied == 0 and st.noops == 60
    absent = np.array([(39 << 32) | v for v in range(40)], np.uint64)
    absent = absent[~np.isin(absent, init)]
    st = g.delete(dev(absent), stats=True)
    assert st.applied == 0
    run_stream(g, ref, V, [("insert", np.repeat(absent[:5], 7)), ("delete", np.repeat(absent[:5], 3))])
    g.close()


@pytest.mark.parametrize("mirror", [False, True])
@pytest.mark.parametrize("kind", ["er", "rmat"])
def test_analytics_match_oracle(kind, mirror):
    """BFS (top-down; with the mirror also bottom-up on large frontiers), CC
    and PageRank (push; with the mirror pull) against the oracle."""
    if kind == "er":
        V = 3000
        edges_t = synth.er_edges(V, 9000, seed=5)
    else:
        u = synth.rmat_unique(12, 16 << 12, seed=6)
        V, edges_t = 1 << 12, u
    e = np.unique(npu64(edges_t))
    g, _ = make(V, e, 32, mirror=mirror)
    for src in (0, 1, V // 2, V - 1):
        assert np.array_equal(g.bfs(src).cpu().numpy(), O.bfs(V, e, src)), src
    assert np.array_equal(g.cc().cpu().numpy().astype(np.uint32), O.cc(V, e))
    x = g.pagerank(iters=10).cpu().numpy()
    want = O.pagerank(V, e, iters=10)
    assert np.max(np.abs(x - want) / want) < PR_RTOL
    # warm start from a non-uniform fp32 vector; out aliases init
    x0 = torch.rand(V, device="cuda", dtype=torch.float32) + 0.1
    x0 /= x0.sum()
    xin = x0.cpu().numpy().astype(np.float64)
    g.pagerank(init=x0, iters=7, damping=0.7, out=x0)
    want = O.pagerank(V, e, x0=xin, iters=7, damping=0.7)
    assert np.max(np.abs(x0.cpu().numpy() - want) / want) < PR_RTOL
    g.close()


def test_analytics_closed_forms():
    from paper_1709_05061_amd import GPMA
    V = 1000
    path = [(i << 32) | (i + 1) for i in range(V - 1)]
    g = GPMA(V, dev(path), leaf_size=16)
    assert list(g.bfs(0).cpu().numpy()) == list(range(V))
    assert list(g.cc().cpu().numpy()) == [0] * V
    x = g.pagerank(iters=10).cpu().numpy()
    assert abs(x.sum() - 1) < 1e-5
    g.close()
    cyc = [(i << 32) | ((i + 1) % V) for i in range(V)]
    g = GPMA(V, dev(cyc), leaf_size=16)
    np.testing.assert_allclose(g.pagerank(iters=10).cpu().numpy(), 1.0 / V, rtol=1e-6)
    g.close()
    g = GPMA(V, dev(np.zeros(0, np.uint64)), leaf_size=16)
    np.testing.assert_allclose(g.pagerank(iters=3).cpu().numpy(), 1.0 / V, rtol=1e-6)
    assert list(g.bfs(5).cpu().numpy()) == [-1] * 5 + [0] + [-1] * (V - 6)
    assert list(g.cc().cpu().numpy()) == list(range(V))
    g.close()


def transpose(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, dtype=np.uint64)
    return (k << np.uint64(32)) | (k >> np.uint64(32))


@pytest.mark.parametrize("kind", ["er", "growth"])
def test_mirror_tracks_every_batch(kind):
    """The dst-major mirror equals an oracle PMA fed the transposed batches;
    PageRank pulled over it matches the fp64 oracle."""
    from paper_1709_05061_amd import GPMA
    if kind == "er":
        V, lf = 1 << 12, 32
        st = synth.er_stream(V, 1 << 15, 1 << 9, 6, seed=21)
        init = npu64(st.initial())
        batches = []
        for t in range(6):
            d, i = st.slide(t, 1 << 9)
            batches += [("delete", npu64(d)), ("insert", npu64(i))]
    else:
        V, lf = 48, 16
        rng = np.random.default_rng(8)
        allk = np.array([(u << 32) | v for u in range(V) for v in range(V)], dtype=np.uint64)
        rng.shuffle(allk)
        init = allk[:30]
        batches = [("insert", allk[30:400]), ("insert", allk[400:1500]), ("delete", allk[:1200]),
                   ("delete", allk[1200:1490])]
    g = GPMA(V, dev(init), leaf_size=lf, mirror=True)
    ref = O.OraclePMA(V, init, lf)
    mref = O.OraclePMA(V, transpose(init), lf)
    m = g.mirror()
    for t, (op, keys) in enumerate(batches):
        say("mirror", kind, t, op)
        getattr(g, op)(dev(keys))
        getattr(ref, op)(keys)
        getattr(mref, op)(transpose(keys))
        edges = check_state(g, ref, V)
        assert np.array_equal(npu64(m.slots()), mref.slots())
        assert np.array_equal(m.row_offsets().cpu().numpy().astype(np.int64), O.row_offsets(mref.slots(), V))
        x = g.pagerank(iters=10).cpu().numpy()
        want = O.pagerank(V, edges, iters=10)
        assert np.max(np.abs(x - want) / want) < PR_RTOL
    g.close()


@pytest.mark.parametrize("mode", ["binned", "binned_gather", "pull", "push"])
def test_spmv_modes_match_oracle_on_rmat(mode):
    """All three SpMV forms (destination bins, pull over the mirror, push with
    atomics) on R-MAT scale 13 against the fp64 oracle."""
    from paper_1709_05061_amd import GPMA
    u = np.unique(npu64(synth.rmat_unique(13, 16 << 13, seed=9)))
    V = 1 << 13
    a = GPMA(V, dev(u), mirror=True, spmv=mode)
    b = GPMA(V, dev(u), mirror=False, spmv=mode if mode != "pull" else "auto")
    say("spmv", mode)
    xa = a.pagerank(iters=10).cpu().numpy()
    xb = b.pagerank(iters=10).cpu().numpy()
    want = O.pagerank(V, u, iters=10)
    assert np.max(np.abs(xa - want) / want) < PR_RTOL
    assert np.max(np.abs(xb - want) / want) < PR_RTOL
    a.close()
    b.close()


@pytest.mark.parametrize("case", ["rmat16", "powerlaw_ragged", "two_level", "many_bins", "rmat16_gather",
                                  "powerlaw_ragged_gather", "many_bins_gather"])
def test_binned_spmv_split_bins_and_ragged_tail(case):
    """Destination bins of 16384 vertices: R-MAT scale 16 puts ~40% of its
    ~1M edges into bin 0, which is cut into several accumulation pieces
    (fp64 atomics between pieces); a power-law graph on 70001 vertices ends
    in a partial bin; 1200001 vertices make 74 bins, so records go through
    coarse bins of 64 bins first (two_level; the last coarse bin partial) or
    are reserved per lane (many_bins).  Warm-started calls after updates too."""
    from paper_1709_05061_amd import GPMA
    form = "binned_coarse" if case == "two_level" else "binned"
    if case.endswith("_gather"):     # the same graphs, edges binned once per call
        form = "binned_gather"
        case = case[: -len("_gather")]
    if case == "rmat16":
        V = 1 << 16
        u = np.unique(npu64(synth.rmat_unique(16, 16 << 16, seed=4)))
    elif case == "powerlaw_ragged":
        V = 70001
        u = np.unique(npu64(synth.powerlaw_edges(V, 600000, seed=6)))
    else:   # 74 bins: coarse bins first (two_level) or per-lane reservations (many_bins)
        V = 1200001
        r = np.unique(npu64(synth.rmat_unique(20, 1 << 21, seed=5)))
        r = r[((r >> np.uint64(32)) < np.uint64(V)) & ((r & np.uint64(0xFFFFFFFF)) < np.uint64(V))]
        u = np.unique(np.concatenate([r, npu64(synth.powerlaw_edges(V, 400000, seed=7))]))
    say("binned", case, V, len(u))
    half = len(u) // 2
    g = GPMA(V, dev(u[:half]), spmv=form)
    ref = O.OraclePMA(V, u[:half], g.leaf_size)
    x = g.pagerank(iters=10).cpu().numpy()
    want = O.pagerank(V, u[:half], iters=10)
    assert np.max(np.abs(x - want) / want) < PR_RTOL
    for t, (op, keys) in enumerate([("insert", u[half:]), ("delete", u[: half // 3])]):
        getattr(g, op)(dev(keys))
        getattr(ref, op)(keys)
        edges = O.edge_keys(ref.slots())
        xin = x.copy()
        x = g.pagerank(init=torch.from_numpy(xin).cuda(), iters=5).cpu().numpy()
        want = O.pagerank(V, edges, x0=xin, iters=5)
        assert np.max(np.abs(x - want) / want) < PR_RTOL, (case, t)
    g.close()


def test_csr_rebuild_comparator_matches_oracle():
    """The rebuild-per-batch CSR comparator holds exactly the oracle's edge set
    (sorted) and its row offsets after every batch, including no-ops,
    repeats, deletes of absent keys and an invalid batch."""
    from paper_1709_05061_amd import CSRRebuild, GpmaError
    V = 1 << 12
    st = synth.er_stream(V, 1 << 15, 1 << 10, 6, seed=21)
    init = npu64(st.initial())
    c = CSRRebuild(V, dev(init))
    ref = O.OraclePMA(V, init, 16)
    for t in range(6):
        d, i = st.slide(t, 1 << 10)
        d = np.concatenate([npu64(d), npu64(synth.random_batch(V, 50, 300 + t))])   # some absent
        i = np.concatenate([npu64(i), npu64(i)[:100]])                             # repeats
        c.delete(dev(d))
        ref.delete(d)
        c.insert(dev(i))
        ref.insert(i)
        e = O.edge_keys(ref.slots())
        assert np.array_equal(npu64(c.keys()), e), t
        want = np.searchsorted(e, np.arange(V + 1, dtype=np.uint64) << np.uint64(32))
        assert np.array_equal(c.row_offsets().cpu().numpy(), want.astype(np.int64)), t
    with pytest.raises(GpmaError):
        c.insert(dev(np.array([(V << 32) | 1], np.uint64)))
    assert np.array_equal(npu64(c.keys()), O.edge_keys(ref.slots()))
    c.close()


@pytest.mark.parametrize("kind", ["rmat", "pieces"])
def test_cc_with_mirror_sampling_path(kind):
    """With a mirror and V >= 4096, CC samples a neighbour per row, picks the
    largest component and sweeps both arrays skipping its rows; labels must
    equal the oracle's (smallest vertex id per weak component): an R-MAT graph
    (one giant component plus isolated vertices) and a union of many small
    directed pieces (no dominant component, long chains)."""
    from paper_1709_05061_amd import GPMA
    if kind == "rmat":
        V = 1 << 14
        e = np.unique(npu64(synth.rmat_unique(14, 4 << 14, seed=13)))
    else:
        V = 6000
        rng = np.random.default_rng(3)
        perm = rng.permutation(V).astype(np.uint64)
        keys = []
        for c0 in range(0, V, 40):            # pieces of 40 vertices: a path with random direction
            blk = perm[c0:c0 + 40]
            for a, b in zip(blk[:-1], blk[1:]):
                keys.append((a << np.uint64(32)) | b if rng.random() < 0.5 else (b << np.uint64(32)) | a)
        e = np.unique(np.array(keys, np.uint64))
    g = GPMA(V, dev(e), mirror=True)
    lab = g.cc().cpu().numpy().astype(np.int64)
    want = O.cc(V, e).astype(np.int64)
    assert np.array_equal(lab, want)
    # again after updates (the sweep must not depend on a fresh handle)
    extra = np.unique(npu64(synth.random_batch(V, 300, 14)))
    g.insert(dev(extra))
    lab = g.cc().cpu().numpy().astype(np.int64)
    assert np.array_equal(lab, O.cc(V, np.union1d(e, extra)).astype(np.int64))
    g.close()


@pytest.mark.parametrize("mirror", [False, True])
def test_degenerate_graphs(mirror):
    """V = 1 (only the self-loop exists), a graph emptied by deletes and
    refilled, zero-length batches inside fused sequences, and the analytics
    on those graphs."""
    from paper_1709_05061_amd import GPMA
    # one vertex
    g = GPMA(1, dev(np.zeros(0, np.uint64)), mirror=mirror)
    ref = O.OraclePMA(1, np.zeros(0, np.uint64), g.leaf_size)
    loop = np.array([0], np.uint64)
    for op in ("insert", "insert", "delete", "delete", "insert"):
        getattr(g, op)(dev(loop))
        getattr(ref, op)(loop)
        assert np.array_equal(npu64(g.slots()), ref.slots())
    assert g.num_edges == 1
    assert np.allclose(g.pagerank(iters=3).cpu().numpy(), [1.0])
    assert g.bfs(0).cpu().numpy().tolist() == [0]
    assert g.cc().cpu().numpy().tolist() == [0]
    g.close()
    # emptied and refilled, with empty batches in a fused sequence
    V = 2000
    e = np.unique(npu64(synth.random_batch(V, 6000, 31)))
    g = GPMA(V, dev(e), leaf_size=16, mirror=mirror)
    ref = O.OraclePMA(V, e, 16)
    z = np.zeros(0, np.uint64)
    ops = [1, 0, 1, 0, 0]
    bs = [e, z, z, e[:10], e]
    g.apply_batches(ops, [dev(b) for b in bs])
    for o, b in zip(ops, bs):
        (ref.delete if o else ref.insert)(b)
    assert np.array_equal(npu64(g.slots()), ref.slots())
    assert g.num_edges == e.size
    g.delete(dev(e))
    ref.delete(e)
    assert g.num_edges == 0 and np.array_equal(npu64(g.slots()), ref.slots())
    x = g.pagerank(iters=5).cpu().numpy()
    assert np.allclose(x, 1.0 / V, rtol=PR_RTOL)
    d = g.bfs(7).cpu().numpy()
    assert d[7] == 0 and (np.delete(d, 7) == -1).all()
    assert np.array_equal(g.cc().cpu().numpy(), np.arange(V))
    g.close()


@pytest.mark.parametrize("mirror", [False, True])
@pytest.mark.parametrize("shape", ["permuted_path", "star_in", "star_out", "many_components"])
def test_cc_contended_unions(shape, mirror):
    """CC applies each union once, by compare-and-swap on roots, in a single
    sweep: shapes that make many threads race on one root (stars), build
    deep trees (a long path whose vertex ids are shuffled), or mix one giant
    component with many small ones (the sampling path skips the giant one)
    must still equal the oracle's union-find."""
    from paper_1709_05061_amd import GPMA
    V = 1 << 14
    rng = np.random.default_rng(["permuted_path", "star_in", "star_out", "many_components"].index(shape) + 40)
    if shape == "permuted_path":
        perm = rng.permutation(V).astype(np.uint64)
        e = (perm[:-1] << np.uint64(32)) | perm[1:]
    elif shape == "star_in":
        leaves = np.arange(1, V, dtype=np.uint64)
        e = (leaves << np.uint64(32)) | np.uint64(V - 1)          # every edge into one hub
    elif shape == "star_out":
        leaves = np.arange(0, V - 1, dtype=np.uint64)
        e = (np.uint64(V // 2) << np.uint64(32)) | leaves          # one hub out to all
        e = e[leaves != np.uint64(V // 2)]
    else:
        big = rng.permutation(V // 2).astype(np.uint64)
        e1 = (big[:-1] << np.uint64(32)) | big[1:]
        small = np.arange(V // 2, V, dtype=np.uint64).reshape(-1, 4)
        e2 = np.concatenate([(small[:, 0] << np.uint64(32)) | small[:, 1],
                             (small[:, 3] << np.uint64(32)) | small[:, 2]])
        e = np.concatenate([e1, e2, rng.choice(e1, 100)])
    e = np.unique(e)
    g, _ = make(V, e, 16, mirror=mirror)
    for _ in range(2):   # repeated calls give the same labels
        assert np.array_equal(g.cc().cpu().numpy().astype(np.uint32), O.cc(V, e))
    g.close()


@pytest.mark.parametrize("V,mirror", [(1 << 26, False), ((1 << 26) + 5, True), ((1 << 26) + 5, False)])
def test_spmv_at_the_bin_limit(V, mirror):
    """The destination-binned SpMV takes up to 4096 bins (V <= 2^26; the
    quiet-bin stage then has the least LDS); one more vertex falls back to
    pull over the mirror or push.  Sparse, skewed graphs at those sizes (the
    67M guards dominate the array) against the fp64 oracle, and BFS/CC."""
    from paper_1709_05061_amd import GPMA
    r = np.unique(npu64(synth.rmat_unique(20, 1 << 21, seed=9)))
    # spread the R-MAT ids over the whole range so every bin sees edges
    src = (r >> np.uint64(32)) * np.uint64(64) + np.uint64(3)
    dst = (r & np.uint64(0xFFFFFFFF)) * np.uint64(64) + np.uint64(1)
    e = np.unique((src << np.uint64(32)) | dst)
    e = e[((e >> np.uint64(32)) < np.uint64(V)) & ((e & np.uint64(0xFFFFFFFF)) < np.uint64(V))]
    say("bin limit", V, mirror, e.size)
    g = GPMA(V, dev(e), mirror=mirror)
    x = g.pagerank(iters=5).cpu().numpy()
    want = O.pagerank(V, e, iters=5)
    assert np.max(np.abs(x - want) / want) < PR_RTOL
    s0 = int(e[0] >> np.uint64(32))
    assert np.array_equal(g.bfs(s0).cpu().numpy(), O.bfs(V, e, s0))
    assert np.array_equal(g.cc().cpu().numpy().astype(np.uint32), O.cc(V, e))
    g.close()
