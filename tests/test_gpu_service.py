"""Streaming service: continuous batching of Poisson edge arrivals with BFS and
PageRank queries admitted into HBM-budgeted slots.  Every query answered in
the mix must equal the same query run alone on the graph version it saw:
BFS exactly, PageRank within 1e-6 (and both against the CPU oracle)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def npu64(t):
    return t.cpu().numpy().view(np.uint64)


def test_service_results_alone_equal_mix():
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd.service import GraphService
    st = synth.rmat_stream(12, 16, seed=3, device="cuda")
    V = st.V
    n_arr = min(20000, st.order.numel() - st.window)
    window = st.initial()
    arrivals = st.order[st.window: st.window + n_arr]
    times = synth.poisson_times(n_arr, 4e4, seed=4)
    nq = 24
    qt = synth.poisson_times(nq, 60.0, seed=5).tolist()
    qt[4:12] = [qt[4]] * 8          # a burst: more queries than slots at once
    kinds = ["bfs" if i % 2 == 0 else "pagerank" for i in range(nq)]
    srcs = synth.uniform_below(torch.arange(nq), 6, V).tolist()
    args = [srcs[i] if kinds[i] == "bfs" else 10 for i in range(nq)]
    svc = GraphService(V, window, leaf_size=16, mirror=True, max_slots=2)
    svc.record = True
    rep = svc.run(times, arrivals, qt, kinds, args, time_limit_s=60)
    s = rep.summary()
    print(s, flush=True)
    assert rep.edges_applied == n_arr
    # the window slid over the whole stream: every arrival was inserted and
    # as many of the oldest edges expired (arrivals are distinct and not in
    # the window, so every update changed the graph)
    assert sum(int(i.numel()) for _, i in svc.batch_log) == n_arr
    assert sum(int(d.numel()) for d, _ in svc.batch_log) == n_arr
    assert rep.updates_applied == 2 * n_arr
    want_final = np.union1d(npu64(window)[n_arr:], npu64(arrivals))
    assert np.array_equal(npu64(svc.g.keys()), want_final)
    assert len(rep.queries) == nq
    assert s["query_slots"] == 2 and rep.max_queue >= 2
    # the edge set at every version, from the batch log
    base = set(int(x) for x in npu64(window))
    versions = {}
    cur = set(base)
    versions[0] = sorted(cur)
    for v, (d, i) in enumerate(svc.batch_log, start=1):
        cur -= set(int(x) for x in d.numpy().view(np.uint64))
        cur |= set(int(x) for x in i.numpy().view(np.uint64))
        versions[v] = sorted(cur)
    for q in rep.queries:
        e = np.array(versions[q.version], dtype=np.uint64)
        alone = GPMA(V, torch.from_numpy(e.view(np.int64)).cuda(), leaf_size=16, mirror=True)
        if q.kind == "bfs":
            a = alone.bfs(q.arg).cpu().numpy()
            assert np.array_equal(q.result, a), (q.qid, q.version)
            assert np.array_equal(q.result, O.bfs(V, e, q.arg))
        else:
            a = alone.pagerank(iters=q.arg).cpu().numpy()
            assert np.max(np.abs(q.result - a) / a) < 1e-6
            want = O.pagerank(V, e, iters=q.arg)
            assert np.max(np.abs(q.result - want) / want) < 1e-6
        alone.close()
    # the live graph equals the last version
    assert np.array_equal(npu64(svc.g.keys()), np.array(versions[len(svc.batch_log)], dtype=np.uint64))
    svc.close()


def test_snapshot_is_frozen_while_updates_continue():
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd.gpma import gpma_bfs, load_library, _HandleView
    import ctypes as C
    lib = load_library()
    V = 2000
    e = np.unique(npu64(synth.random_batch(V, 20000, 7)))
    g = GPMA(V, torch.from_numpy(e.view(np.int64)).cuda(), leaf_size=16, mirror=True)
    h = C.c_void_p()
    s = torch.cuda.current_stream()
    assert lib.gpma_snapshot(g.h, C.byref(h), C.c_void_p(s.cuda_stream)) == 0
    before = npu64(_HandleView(h, V).slots())
    g.insert(synth.random_batch(V, 30000, 8).cuda())     # grows: the live array resizes
    after = npu64(_HandleView(h, V).slots())
    assert np.array_equal(before, after)
    assert g.capacity != len(after) or not np.array_equal(npu64(g.slots()), after)
    d = torch.empty(V, dtype=torch.int32, device="cuda")
    gpma_bfs(h, 0, d)
    assert np.array_equal(d.cpu().numpy(), O.bfs(V, e, 0))
    assert lib.gpma_insert_batch(h, C.c_void_p(synth.random_batch(V, 5, 9).cuda().data_ptr()), 5,
                                 C.c_void_p(s.cuda_stream), None) == -1
    assert lib.gpma_snapshot_refresh(g.h, h, C.c_void_p(s.cuda_stream)) == 0
    assert np.array_equal(npu64(_HandleView(h, V).slots()), npu64(g.slots()))
    lib.gpma_destroy(h)
    g.close()


def test_service_budget_admits_growth_by_giving_up_slots():
    """One HBM budget for the graph and the query slots: the window only
    grows (no expiry), so the array resizes; under a budget that holds the
    grown graph but not all slots beside it, a refused update batch waits
    while idle slots give their memory up, queries queue for the slots that
    are left, and every answer still equals the oracle on the version it
    saw."""
    from paper_1709_05061_amd.service import GraphService
    st = synth.rmat_stream(13, 16, seed=8, device="cuda")
    V = st.V
    window = st.order[: st.window // 8]
    arrivals = st.order[st.window // 8: st.window // 8 + 40000]
    times = torch.zeros(arrivals.numel(), dtype=torch.float64)      # all arrived: back-to-back steps
    nq = 30
    qt = [0.0] * nq
    kinds = ["bfs" if i % 2 == 0 else "pagerank" for i in range(nq)]
    srcs = synth.uniform_below(torch.arange(nq), 9, V).tolist()
    args = [srcs[i] if kinds[i] == "bfs" else 10 for i in range(nq)]
    # a dry run with room for everything measures the peak of one slot beside the grown graph
    probe = GraphService(V, window, leaf_size=16, mirror=True, max_slots=1, max_batch=1 << 12, expire=False,
                         hbm_budget_bytes=1 << 36)
    probe.run(times, arrivals, [], [], [], time_limit_s=60)
    peak = probe.alloc.peak_bytes
    probe.close()
    svc = GraphService(V, window, leaf_size=16, mirror=True, max_slots=3, max_batch=1 << 12, expire=False,
                       hbm_budget_bytes=peak)
    svc.record = True
    slots0 = sum(1 for s in svc.slots if s is not None)
    rep = svc.run(times, arrivals, qt, kinds, args, time_limit_s=120)
    s = rep.summary()
    print(s, flush=True)
    assert slots0 >= 2, slots0
    assert rep.update_waits >= 1 and rep.slots_given_up >= 1
    assert rep.max_queue >= nq - slots0
    assert len(rep.queries) == nq
    assert rep.peak_bytes <= peak
    want_final = np.unique(np.concatenate([npu64(window), npu64(arrivals)]))
    assert np.array_equal(npu64(svc.g.keys()), want_final)
    cur = set(int(x) for x in npu64(window))
    versions = {0: sorted(cur)}
    for v, (d, i) in enumerate(svc.batch_log, start=1):
        assert d.numel() == 0
        cur |= set(int(x) for x in i.numpy().view(np.uint64))
        versions[v] = sorted(cur)
    for q in rep.queries:
        e = np.array(versions[q.version], dtype=np.uint64)
        if q.kind == "bfs":
            assert np.array_equal(q.result, O.bfs(V, e, q.arg)), (q.qid, q.version)
        else:
            want = O.pagerank(V, e, iters=q.arg)
            assert np.max(np.abs(q.result - want) / want) < 1e-6
    svc.close()
