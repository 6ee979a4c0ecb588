"""Parity in the shapes of the other workloads, slot for slot against the
sequential oracle.

R-MAT scale 20 (edge factor 16, window = the first half of the distinct
edges): slides of 2^16 and then of 2^20 deletes + inserts; at this size the
2^20 batches climb through the workgroup tier and the host-driven device
tier.  After every slide the raw slot arrays equal the oracle's, and BFS
from 8 sources with out-edges, CC and 10-step PageRank equal the oracle's
analytics.  Plain path (each batch's per-level merge counts against the
oracle's merge log) and fused path (dst-major mirror, learned locator; the
mirror against an oracle of the transposed edges).

Power-law shape (out-degree exponent 2.1, window = first half): uneven
slides of log-uniform size 2^6..2^14 fused in three calls (mirror, learned
locator), array and mirror against the oracle after each call."""
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


def host(t):
    return t.cpu().numpy().view(np.uint64)


def transpose(k):
    return ((k & np.uint64(0xFFFFFFFF)) << np.uint64(32)) | (k >> np.uint64(32))


def same_slots(h, ref, what):
    got = host(h.slots())
    want = ref.slots()
    assert got.size == want.size, (what, got.size, want.size)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%s: %d slots differ, first at %s" % (what, bad.size, bad[:5])


@pytest.mark.timeout(900)
def test_rmat20_slides_2e16_and_2e20():
    from paper_1709_05061_amd import GPMA
    from test_gpu_pma import check_merge_log
    st = synth.rmat_stream(20, 16, seed=2, device="cuda")
    V = st.V
    init = host(torch.sort(st.initial())[0])
    plain = GPMA(V, st.initial(), leaf_size=32)
    fused = GPMA(V, st.initial(), leaf_size=32, mirror=True, learned=True)
    ref = O.OraclePMA(V, init, 32)
    mref = O.OraclePMA(V, np.sort(transpose(init)), 32)
    same_slots(plain, ref, "create")
    say("R-MAT 20: window", st.window, "capacity", ref.capacity)
    rng = np.random.default_rng(20)
    t0 = 0
    for t, b in enumerate([1 << 16, 1 << 16, 1 << 20, 1 << 20]):
        d, i = st.order[t0:t0 + b], st.order[st.window + t0: st.window + t0 + b]
        t0 += b
        say("slide", t, "b", b)
        for op, keys in (("delete", d), ("insert", i)):
            cap0 = ref.capacity
            s = getattr(plain, op)(keys, stats=True)
            getattr(ref, op)(host(keys))
            getattr(mref, op)(transpose(host(keys)))
            assert s.applied == ref.last_applied() == b
            check_merge_log(s, ref, 32, cap0)
        fs = fused.apply_batches([1, 0], [d, i])
        assert fs.applied == 2 * b
        same_slots(plain, ref, "plain slide %d" % t)
        same_slots(fused, ref, "fused slide %d" % t)
        same_slots(fused.mirror(), mref, "mirror slide %d" % t)
        edges = O.edge_keys(ref.slots())
        deg = np.bincount((edges >> np.uint64(32)).astype(np.int64), minlength=V)
        srcs = rng.choice(np.nonzero(deg)[0], 8, replace=False)
        for src in srcs:
            want = O.bfs(V, edges, int(src))
            assert np.array_equal(plain.bfs(int(src)).cpu().numpy(), want), src
            assert np.array_equal(fused.bfs(int(src)).cpu().numpy(), want), src
        want = O.cc(V, edges)
        assert np.array_equal(plain.cc().cpu().numpy().astype(np.uint32), want)
        assert np.array_equal(fused.cc().cpu().numpy().astype(np.uint32), want)
        want = O.pagerank(V, edges, iters=10)
        for g in (plain, fused):
            x = g.pagerank(iters=10).cpu().numpy()
            assert np.max(np.abs(x - want) / want) < PR_RTOL
    plain.close()
    fused.close()


@pytest.mark.timeout(600)
def test_powerlaw_uneven_slides_fused():
    from paper_1709_05061_amd import GPMA
    V = 1 << 17
    e = synth.powerlaw_edges(V, 1 << 21, seed=30, device="cuda")
    st = synth.Stream(V, e, e.numel() // 2)
    init = host(torch.sort(st.initial())[0])
    g = GPMA(V, st.initial(), leaf_size=32, mirror=True, learned=True)
    ref = O.OraclePMA(V, init, 32)
    mref = O.OraclePMA(V, np.sort(transpose(init)), 32)
    sizes = synth.loguniform_sizes(30, 6, 14, 31)
    ops, bs, pos = [], [], 0
    for b in sizes:
        ops += [1, 0]
        bs += [st.order[pos:pos + b], st.order[st.window + pos: st.window + pos + b]]
        pos += b
    say("power-law: window", st.window, "slides", len(sizes), "updates", 2 * pos)
    for c0, c1 in ((0, 14), (14, 40), (40, len(ops))):
        s = g.apply_batches(ops[c0:c1], bs[c0:c1])
        applied = 0
        for op, keys in zip(ops[c0:c1], bs[c0:c1]):
            (ref.delete if op else ref.insert)(host(keys))
            (mref.delete if op else mref.insert)(transpose(host(keys)))
            applied += ref.last_applied()
        assert s.applied == applied
        same_slots(g, ref, "array after batches %d..%d" % (c0, c1))
        same_slots(g.mirror(), mref, "mirror after batches %d..%d" % (c0, c1))
    g.close()
