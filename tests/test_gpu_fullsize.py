"""Parity at the headline size, in the configuration the benchmark times:
R-MAT scale 24, edge factor 16 (all distinct edges of 2^28 draws, ~2.6e8,
a 2^29-slot array), dst-major mirror, learned locator, fused batching with
1024-key sort tiles and no device levels above the leaves; two slides of
2^16 deletes + 2^16 inserts.  The sequential layout oracle replays the same
two slides (a few seconds per batch at this size, its work is linear in the
capacity), so the raw slot arrays of the array and of the mirror are
compared byte for byte; the oracle's analytics (plain C) compare PageRank,
BFS and CC on every vertex; the edge set is compared with the stream's
window after the slides and the degrees with a count of the exported
edges."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
def test_fullsize_rmat24_bench_configuration():
    from paper_1709_05061_amd import GPMA
    b = 1 << 16
    say("generating R-MAT scale 24")
    st = synth.rmat_full_stream(24, 16, 1 << 20, 1, device="cuda")
    V = st.V
    g = GPMA(V, st.initial(), mirror=True, learned=True, sort_tile=1024, fused_levels=0)
    assert g.capacity == 1 << 29
    for t in range(2):
        d, i = st.slide(t, b)
        s = g.apply_batches([1, 0], [d, i])
        assert s.applied == 2 * b, (t, s)
    torch.cuda.synchronize()
    say("slides applied; replaying them through the layout oracle")
    lf = g.leaf_size
    for name, h, tr in (("array", g, False), ("mirror", g.mirror(), True)):
        def t(k):   # device keys, transposed for the mirror, as host uint64
            k = ((k & 0xFFFFFFFF) << 32) | (k >> 32) if tr else k
            return k.cpu().numpy().view(np.uint64)
        # the initial set handed over sorted (a set: the order of the input
        # does not change what the oracle builds, only how long its sort takes)
        k0 = st.initial()
        k0 = ((k0 & 0xFFFFFFFF) << 32) | (k0 >> 32) if tr else k0
        ref = O.OraclePMA(V, torch.sort(k0)[0].cpu().numpy().view(np.uint64), lf)
        del k0
        for s_ in range(2):
            d, i = st.slide(s_, b)
            ref.delete(t(d))
            ref.insert(t(i))
        want = ref.slots()
        del ref
        got = h.slots().cpu().numpy().view(np.uint64)
        assert got.size == want.size
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, "%s: %d slots differ, first at %s" % (name, bad.size, bad[:5])
        say(name, "slot for slot equal to the oracle")
        del want, got
    say("comparing the edge set")
    keys = g.keys()
    want = torch.sort(st.order[2 * b: st.window + 2 * b])[0]
    assert torch.equal(keys, want)
    m = g.mirror()
    tr = ((keys & 0xFFFFFFFF) << 32) | (keys >> 32)
    assert torch.equal(m.keys(), torch.sort(tr)[0])
    del want, tr
    edges = keys.cpu().numpy().view(np.uint64)
    del keys
    torch.cuda.empty_cache()
    assert np.array_equal(g.degrees().cpu().numpy().astype(np.int64),
                          np.bincount((edges >> np.uint64(32)).astype(np.int64), minlength=V))
    say("slot invariants")
    slots = g.slots().cpu().numpy().view(np.uint64)
    O.check_invariants(slots, g.leaf_size, V)
    assert np.array_equal(g.row_offsets().cpu().numpy().astype(np.int64), O.row_offsets(slots, V))
    assert np.array_equal(g.leaf_counts().cpu().numpy().astype(np.int64), O.leaf_counts(slots, g.leaf_size))
    assert np.array_equal(g.pivots().cpu().numpy().view(np.uint64), O.leaf_pivots(slots, g.leaf_size))
    del slots
    say("PageRank")
    x0 = torch.rand(V, device="cuda", dtype=torch.float32) + 0.1
    x0 /= x0.sum()
    xin = x0.cpu().numpy().astype(np.float64)
    x = g.pagerank(init=x0, iters=10).cpu().numpy()
    ref = O.pagerank(V, edges, x0=xin, iters=10)
    assert np.max(np.abs(x - ref) / ref) < 1e-6
    say("BFS")
    deg = np.bincount((edges >> np.uint64(32)).astype(np.int64), minlength=V)
    for src in (0, int(np.nonzero(deg)[0][-1])):
        assert np.array_equal(g.bfs(src).cpu().numpy(), O.bfs(V, edges, src)), src
    say("CC")
    assert np.array_equal(g.cc().cpu().numpy().astype(np.uint32), O.cc(V, edges))
    g.close()
