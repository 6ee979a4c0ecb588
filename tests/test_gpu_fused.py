"""Fused batching (HIP-graph replay of uneven batch sequences) equals the
plain per-batch path slot for slot, including batches that climb above the
captured levels and resize the root, graphs replayed many times with eager
plain batches in between, and the mirror."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(keys):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).view(np.int64)).cuda()


def npu64(t):
    return t.cpu().numpy().view(np.uint64)


def check_pivots(g):
    """The locate's pivot array equals each leaf's first slot, mark cleared
    (array and mirror)."""
    for h in ((g, g.mirror()) if g.mirror() is not None else (g,)):
        assert np.array_equal(npu64(h.pivots()), O.leaf_pivots(npu64(h.slots()), h.leaf_size))


def make_sequence(V, live, n, seed):
    """n uneven batches (sizes log-uniform 2^3..2^12): inserts of random keys,
    deletes of live keys plus absent ones; one sorted run and one large
    insert that forces a resize."""
    rng = np.random.default_rng(seed)
    live = set(int(x) for x in live)
    ops, bs = [], []
    for t in range(n):
        size = int(2 ** rng.uniform(3, 12))
        if t == n // 3:      # sorted run into one corner: climbs levels
            u = int(rng.integers(0, V))
            keys = np.array([(u << 32) | v for v in range(V)][:size], np.uint64)
            op = 0
        elif t == 2 * n // 3:    # large insert: the root doubles
            keys = np.array([(int(a) << 32) | int(b) for a, b in
                             zip(rng.integers(0, V, 4 * len(live) + 64), rng.integers(0, V, 4 * len(live) + 64))],
                            np.uint64)
            op = 0
        elif rng.random() < 0.5 or len(live) < 2 * size:
            keys = np.array([(int(a) << 32) | int(b) for a, b in
                             zip(rng.integers(0, V, size), rng.integers(0, V, size))], np.uint64)
            op = 0
        else:
            pool = np.array(sorted(live), np.uint64)
            keys = np.concatenate([pool[rng.choice(pool.size, size, replace=False)],
                                   np.array([(int(V - 1) << 32) | int(rng.integers(0, V))], np.uint64)])
            op = 1
        keys = np.concatenate([keys, keys[: max(1, keys.size // 10)]])   # repeats
        if op == 0:
            live |= set(int(x) for x in keys)
        else:
            live -= set(int(x) for x in keys)
        ops.append(op)
        bs.append(keys)
    return ops, bs


@pytest.mark.parametrize("mirror,direct,tile,levels", [(False, False, 0, 1), (True, False, 0, 2),
                                                       (False, True, 512, 0), (True, True, 2048, 3),
                                                       (True, True, 1024, 0)])
def test_fused_equals_plain(mirror, direct, tile, levels):
    """Fused sequences (graph replay or direct enqueue, every sort tile)
    equal the plain per-batch path and the oracle."""
    from paper_1709_05061_amd import GPMA
    V, lf = 512, 16
    init = np.unique(npu64(synth.random_batch(V, 6000, 3)))
    ops, bs = make_sequence(V, init, 36, seed=5)
    plain = GPMA(V, dev(init), leaf_size=lf, mirror=mirror)
    fused = GPMA(V, dev(init), leaf_size=lf, mirror=mirror, fused_direct=direct, sort_tile=tile,
                 fused_levels=levels)
    ref = O.OraclePMA(V, init, lf)
    cuts = [0, 5, 6, 20, 36]
    for c in range(len(cuts) - 1):
        lo, hi = cuts[c], cuts[c + 1]
        say("fused call", lo, hi, "mirror", mirror, "direct", direct, "tile", tile, "levels", levels)
        for i in range(lo, hi):
            (plain.delete if ops[i] else plain.insert)(dev(bs[i]))
            (ref.delete if ops[i] else ref.insert)(bs[i])
        st = fused.apply_batches(ops[lo:hi], [dev(b) for b in bs[lo:hi]])
        assert np.array_equal(npu64(fused.slots()), npu64(plain.slots())), (lo, hi)
        assert np.array_equal(npu64(fused.slots()), ref.slots())
        check_pivots(fused)
        assert fused.num_edges == plain.num_edges
        assert np.array_equal(fused.degrees().cpu().numpy(), plain.degrees().cpu().numpy())
        assert np.array_equal(fused.row_offsets().cpu().numpy(), plain.row_offsets().cpu().numpy())
        if mirror:
            assert np.array_equal(npu64(fused.mirror().slots()), npu64(plain.mirror().slots()))
        # an eager plain batch between graph replays, on both handles
        extra = npu64(synth.random_batch(V, 37, 100 + c))
        plain.insert(dev(extra))
        fused.insert(dev(extra))
        ref.insert(extra)
        assert np.array_equal(npu64(fused.slots()), npu64(plain.slots()))
    plain.close()
    fused.close()


@pytest.mark.parametrize("direct", [False, True])
def test_fused_replays_many_batches_same_class(direct):
    """Many replays of the same cached graphs (one size class)."""
    from paper_1709_05061_amd import GPMA
    V = 1 << 12
    st = synth.er_stream(V, 1 << 15, 700, 24, seed=9)
    plain = GPMA(V, st.initial().cuda(), leaf_size=32, sort_tile=512)
    fused = GPMA(V, st.initial().cuda(), leaf_size=32, fused_direct=direct)
    ops, bs = [], []
    for t in range(24):
        d, i = st.slide(t, 700)
        d, i = d.cuda(), i.cuda()
        ops += [1, 0]
        bs += [d, i]
        plain.delete(d)
        plain.insert(i)
    for rep in range(3):
        lo, hi = 16 * rep, 16 * (rep + 1)
        s = fused.apply_batches(ops[lo:hi], bs[lo:hi])
        assert s.applied == 700 * (hi - lo)
    assert np.array_equal(npu64(fused.slots()), npu64(plain.slots()))
    plain.close()
    fused.close()


def test_fused_invalid_key_stops_at_that_batch():
    from paper_1709_05061_amd import GPMA, GpmaError
    from paper_1709_05061_amd.gpma import gpma_apply_batches
    V = 300
    init = np.unique(npu64(synth.random_batch(V, 2000, 1)))
    g = GPMA(V, dev(init), leaf_size=16)
    ref = O.OraclePMA(V, init, 16)
    good = [npu64(synth.random_batch(V, 50, 10 + i)) for i in range(4)]
    bad = np.array([(V << 32) | 1], np.uint64)
    seq = [good[0], good[1], bad, good[2]]
    with pytest.raises(GpmaError) as ei:
        gpma_apply_batches(g.h, [0, 0, 0, 0], [dev(b) for b in seq])
    assert ei.value.code == -1
    ref.insert(good[0])
    ref.insert(good[1])
    assert np.array_equal(npu64(g.slots()), ref.slots())
    g.close()


@pytest.mark.parametrize("mirror", [False, True])
def test_fused_windows_invalid_batch_then_more_calls(mirror):
    """40 batches in one call (windows of 8, 16, ... batches sorted together),
    an invalid key in batch 13: batches 0..12 stand, the call reports it, and
    later calls (new windows, new generations) are unaffected by the stale
    error flag."""
    from paper_1709_05061_amd import GPMA, GpmaError
    from paper_1709_05061_amd.gpma import gpma_apply_batches
    V, lf = 700, 16
    init = np.unique(npu64(synth.random_batch(V, 5000, 2)))
    ops, bs = make_sequence(V, init, 40, seed=11)
    bad = bs[13].copy()
    bad[len(bad) // 2] = np.uint64((V << 32) | 3)
    seq = bs[:13] + [bad] + bs[14:]
    g = GPMA(V, dev(init), leaf_size=lf, mirror=mirror)
    ref = O.OraclePMA(V, init, lf)
    with pytest.raises(GpmaError) as ei:
        gpma_apply_batches(g.h, ops, [dev(b) for b in seq])
    assert ei.value.code == -1
    for i in range(13):
        (ref.delete if ops[i] else ref.insert)(bs[i])
    assert np.array_equal(npu64(g.slots()), ref.slots())
    # the rest of the sequence, valid, in two more calls
    g.apply_batches(ops[13:30], [dev(b) for b in bs[13:30]])
    g.apply_batches(ops[30:], [dev(b) for b in bs[30:]])
    for i in range(13, 40):
        (ref.delete if ops[i] else ref.insert)(bs[i])
    assert np.array_equal(npu64(g.slots()), ref.slots())
    if mirror:
        t = lambda a: (a << np.uint64(32)) | (a >> np.uint64(32))
        mref = O.OraclePMA(V, t(init), lf)
        for i in range(40):
            (mref.delete if ops[i] else mref.insert)(t(bs[i]))
        assert np.array_equal(npu64(g.mirror().slots()), mref.slots())
    g.close()


@pytest.mark.parametrize("n_extra,lib_streams", [(0, False), (1, False), (2, False), (3, False), (5, False),
                                                 (0, True), (3, True)])
def test_fused_mirror_under_other_streams(n_extra, lib_streams):
    """With a mirror the fused pipelines run in one of two arrangements: the
    array's on the caller's stream and the mirror's on a handle stream that a
    probe found running beside it (pairing 1), or both on handle streams
    forked from and joined to the caller's (pairing 0, forced here by
    GPMA_FLAG_FUSED_LIB_STREAMS and taken when no handle stream runs
    beside the caller's).  Other live streams in the process change which
    hardware queues the streams sit on; the result must not change: fused
    equals plain on the array and the mirror, also when the caller works on
    a non-default stream."""
    from paper_1709_05061_amd import GPMA
    extra = []
    for _ in range(n_extra):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            torch.zeros(1, device="cuda")
        extra.append(s)
    V, lf = 700, 16
    init = np.unique(npu64(synth.random_batch(V, 8000, 7)))
    ops, bs = make_sequence(V, init, 24, seed=11 + n_extra)
    plain = GPMA(V, dev(init), leaf_size=lf, mirror=True)
    fused = GPMA(V, dev(init), leaf_size=lf, mirror=True, fused_levels=1, lib_streams=lib_streams)
    caller = torch.cuda.Stream() if n_extra % 2 else torch.cuda.current_stream()
    say("fused under", n_extra, "extra streams, caller stream", caller, "library streams", lib_streams)
    for lo, hi in ((0, 10), (10, 11), (11, 24)):
        for i in range(lo, hi):
            (plain.delete if ops[i] else plain.insert)(dev(bs[i]))
        keys = [dev(b) for b in bs[lo:hi]]
        torch.cuda.synchronize()
        with torch.cuda.stream(caller):
            fused.apply_batches(ops[lo:hi], keys)
        torch.cuda.synchronize()
        assert np.array_equal(npu64(fused.slots()), npu64(plain.slots())), (lo, hi)
        assert np.array_equal(npu64(fused.mirror().slots()), npu64(plain.mirror().slots())), (lo, hi)
        assert fused.num_edges == plain.num_edges
    pairing = fused.fused_pairing(caller)
    say("pairing", pairing)
    if lib_streams:
        assert pairing == 0
    else:
        assert pairing in (0, 1)
    plain.close()
    fused.close()


def _window_case(kind, seed):
    """(V, leaf size, initial keys, ops, batches) of one window-sort case."""
    rng = np.random.default_rng(seed)

    def rand(V, n):
        return (rng.integers(0, V, n).astype(np.uint64) << np.uint64(32)) | rng.integers(0, V, n).astype(np.uint64)

    if kind == "duplicates":
        # one key repeated past what a bucket sorts in LDS, in an insert and
        # in a delete window: the bucket takes the global-memory path
        V = 1 << 12
        init = np.unique(rand(V, 1 << 15))
        hot = np.uint64((7 << 32) | 9)
        live_hot = init[len(init) // 2]
        ops = [0, 1, 0, 1]
        bs = [np.concatenate([np.full(9000, hot, np.uint64), rand(V, 3000)]),
              np.concatenate([np.full(5000, live_hot, np.uint64), init[:2000]]),
              np.full(6000, hot, np.uint64),
              np.concatenate([rand(V, 700), np.full(4500, hot, np.uint64)])]
        return V, 16, init, ops, bs
    if kind == "tiny":
        V = 1 << 10
        init = np.unique(rand(V, 1 << 13))
        ops = [0, 1, 0, 0, 1, 0, 1]
        bs = [rand(V, 1), init[:1], rand(V, 2), rand(V, 3), init[5:8], np.zeros(0, np.uint64), rand(V, 1)]
        return V, 16, init, ops, bs
    # "large": windows of 2^20 keys (the splitter sort's largest) and of
    # 1.5 * 2^20 keys (the radix sort)
    V = 1 << 16
    init = np.unique(rand(V, 1 << 20))
    ops = [1, 0, 0, 1, 0]
    half = 1 << 19
    bs = [init[rng.choice(init.size, half, replace=False)], rand(V, half),
          rand(V, half), init[rng.choice(init.size, half, replace=False)], rand(V, half)]
    return V, 32, init, ops, bs


@pytest.mark.parametrize("kind", ["duplicates", "tiny", "large"])
@pytest.mark.parametrize("window_sort", ["splitter", "radix"])
def test_window_sorts_agree_with_the_oracle(kind, window_sort):
    """Both sorts of a fused window's keys (the splitter sort, and the radix
    sort it replaces) give the oracle's slots: repeated keys beyond a bucket's
    LDS capacity, windows of 1-3 keys and an empty batch, and windows at and
    above the splitter sort's 2^20-key limit."""
    from paper_1709_05061_amd import GPMA
    V, lf, init, ops, bs = _window_case(kind, 31)
    mirror = kind != "large"
    g = GPMA(V, dev(init), leaf_size=lf, mirror=mirror, window_sort=window_sort)
    ref = O.OraclePMA(V, init, lf)
    cuts = [0, 2, len(ops)]
    for c in range(len(cuts) - 1):
        lo, hi = cuts[c], cuts[c + 1]
        say(kind, window_sort, "batches", lo, hi, [b.size for b in bs[lo:hi]])
        st = g.apply_batches(ops[lo:hi], [dev(b) for b in bs[lo:hi]])
        applied = 0
        for i in range(lo, hi):
            (ref.delete if ops[i] else ref.insert)(bs[i])
            applied += ref.last_applied()
        assert st.applied == applied, (kind, window_sort, lo, hi)
        assert np.array_equal(npu64(g.slots()), ref.slots()), (kind, window_sort, lo, hi)
        check_pivots(g)
        if mirror:
            k = g.keys()
            tr = ((k & 0xFFFFFFFF) << 32) | (k >> 32)
            assert torch.equal(g.mirror().keys(), torch.sort(tr)[0])
    assert g.num_edges + V == ref.size   # the oracle counts the V guards
    g.close()


@pytest.mark.parametrize("learned,lazy", [(False, False), (True, False), (False, True)])
def test_paired_windows_equal_plain(learned, lazy):
    """With a mirror and no device level above the leaves, both sides of a
    window run each step in one launch (paired windows).  Uneven sequences
    with batches that climb above the leaves, a resize, repeats and absent
    deletes give the plain path's and the oracle's slots, array and mirror;
    the sides stop at different batches and pair again afterwards."""
    from paper_1709_05061_amd import GPMA
    V, lf = 512, 16
    init = np.unique(npu64(synth.random_batch(V, 6000, 13)))
    ops, bs = make_sequence(V, init, 40, seed=15)
    kw = dict(leaf_size=lf, mirror=True, learned=learned, lazy_delete=lazy)
    plain = GPMA(V, dev(init), **kw)
    fused = GPMA(V, dev(init), fused_levels=0, **kw)
    cuts = [0, 4, 5, 19, 40]
    for c in range(len(cuts) - 1):
        lo, hi = cuts[c], cuts[c + 1]
        say("paired call", lo, hi, "learned", learned, "lazy", lazy)
        applied = noops = 0
        for i in range(lo, hi):
            sp = (plain.delete if ops[i] else plain.insert)(dev(bs[i]), stats=True)
            applied += sp.applied
            noops += sp.noops
        st = fused.apply_batches(ops[lo:hi], [dev(b) for b in bs[lo:hi]])
        # the call's statistics (written by the device into the pinned results
        # for paired windows) agree with the plain batches'
        assert (st.applied, st.noops) == (applied, noops), (lo, hi, st, applied, noops)
        assert np.array_equal(npu64(fused.slots()), npu64(plain.slots())), (lo, hi)
        assert np.array_equal(npu64(fused.mirror().slots()), npu64(plain.mirror().slots())), (lo, hi)
        check_pivots(fused)
        assert fused.num_edges == plain.num_edges
        assert np.array_equal(fused.degrees().cpu().numpy(), plain.degrees().cpu().numpy())
    if not lazy:
        ref = O.OraclePMA(V, init, lf)
        for o, b in zip(ops, bs):
            (ref.delete if o else ref.insert)(b)
        assert np.array_equal(npu64(fused.slots()), ref.slots())
    plain.close()
    fused.close()
