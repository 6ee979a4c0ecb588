"""Device memory through the caller's allocator, and GPMA_ENOMEM that changes
nothing.  An allocator that refuses every request from a chosen point on
makes the first root resize (growth by an insert batch, halving by a delete
batch, a fused sequence) fail: the call returns GPMA_ENOMEM and the slot
array, leaf counts, row offsets, degrees, edge count, capacity and mirror are
byte-identical to before; allowed again, the same batch gives the oracle's
layout slot for slot."""
import sys

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(keys):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).view(np.int64)).cuda()


def npu64(t):
    return t.cpu().numpy().view(np.uint64)


def state(g):
    s = [npu64(g.slots()), g.leaf_counts().cpu().numpy(), g.row_offsets().cpu().numpy(),
         g.degrees().cpu().numpy(), g.num_edges, g.capacity]
    m = g.mirror()
    if m is not None:
        s += [npu64(m.slots()), m.leaf_counts().cpu().numpy(), m.num_edges, m.capacity]
    return s


def same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y)
        else:
            assert x == y


def refusing_allocator():
    from paper_1709_05061_amd.gpma import TorchAllocator

    class Refusing(TorchAllocator):
        refuse = False
        refused = 0

        def allow(self, nbytes):
            if self.refuse:
                self.refused += 1
                return False
            return True
    return Refusing()


def all_keys(V, seed):
    rng = np.random.default_rng(seed)
    k = np.array([(u << 32) | v for u in range(V) for v in range(V)], dtype=np.uint64)
    rng.shuffle(k)
    return k


@pytest.mark.parametrize("mirror", [False, True])
def test_enomem_on_growth_changes_nothing(mirror):
    from paper_1709_05061_amd import GPMA, GpmaError
    from paper_1709_05061_amd.gpma import GPMA_ENOMEM
    V, lf = 64, 16
    k = all_keys(V, 1)
    al = refusing_allocator()
    g = GPMA(V, dev(k[:300]), leaf_size=lf, mirror=mirror, allocator=al)
    ref = O.OraclePMA(V, k[:300], lf)
    g.insert(dev(k[300:340]))
    ref.insert(k[300:340])
    assert np.array_equal(npu64(g.slots()), ref.slots())
    batch = k[340:2000]
    cap0 = ref.capacity
    probe = O.OraclePMA(V, O.edge_keys(ref.slots()), lf)
    probe.insert(batch)
    assert probe.capacity > cap0            # this batch resizes the root
    before = state(g)
    al.refuse = True
    say("growth with a refusing allocator, mirror", mirror)
    with pytest.raises(GpmaError) as ei:
        g.insert(dev(batch))
    assert ei.value.code == GPMA_ENOMEM and al.refused > 0
    al.refuse = False
    same(before, state(g))
    g.insert(dev(batch))
    ref.insert(batch)
    assert ref.capacity > cap0
    assert np.array_equal(npu64(g.slots()), ref.slots())
    if mirror:
        mref = O.OraclePMA(V, np.sort((k[:2000] >> np.uint64(32)) | (k[:2000] << np.uint64(32))), lf)
        assert np.array_equal(O.edge_keys(npu64(g.mirror().slots())), O.edge_keys(mref.slots()))
    assert g.allocated_bytes == al.held_bytes > 0
    g.close()
    assert al.held_bytes == 0


def test_enomem_on_halving_changes_nothing():
    from paper_1709_05061_amd import GPMA, GpmaError
    from paper_1709_05061_amd.gpma import GPMA_ENOMEM
    V, lf = 64, 16
    k = all_keys(V, 2)
    al = refusing_allocator()
    g = GPMA(V, dev(k[:3000]), leaf_size=lf, mirror=True, allocator=al)
    ref = O.OraclePMA(V, k[:3000], lf)
    g.delete(dev(k[:10]))
    ref.delete(k[:10])
    batch = k[10:2600]
    cap0 = ref.capacity
    before = state(g)
    al.refuse = True
    say("halving with a refusing allocator")
    with pytest.raises(GpmaError) as ei:
        g.delete(dev(batch))
    assert ei.value.code == GPMA_ENOMEM
    al.refuse = False
    same(before, state(g))
    g.delete(dev(batch))
    ref.delete(batch)
    assert ref.capacity < cap0
    assert np.array_equal(npu64(g.slots()), ref.slots())
    g.close()


def test_enomem_in_fused_sequence_applies_nothing():
    from paper_1709_05061_amd import GPMA, GpmaError
    from paper_1709_05061_amd.gpma import GPMA_ENOMEM, gpma_apply_batches
    V, lf = 64, 16
    k = all_keys(V, 3)
    al = refusing_allocator()
    g = GPMA(V, dev(k[:200]), leaf_size=lf, mirror=True, allocator=al)
    ref = O.OraclePMA(V, k[:200], lf)
    ops = [0, 0, 1, 0]
    batches = [k[200:400], k[400:1500], k[100:300], k[1500:3000]]
    before = state(g)
    al.refuse = True
    say("fused sequence with a refusing allocator")
    with pytest.raises(GpmaError) as ei:
        g.apply_batches(ops, [dev(b) for b in batches])
    assert ei.value.code == GPMA_ENOMEM
    al.refuse = False
    same(before, state(g))
    st, done = gpma_apply_batches(g.h, ops, [dev(b) for b in batches])
    assert done == 4
    for op, b in zip(ops, batches):
        (ref.delete if op else ref.insert)(b)
    assert np.array_equal(npu64(g.slots()), ref.slots())
    g.close()


def test_library_allocator_and_torch_allocator_agree():
    """The same stream through hipMalloc (allocator=False) and through torch's
    caching allocator: identical layouts; the handle's byte count follows
    the arrays it holds."""
    from paper_1709_05061_amd import GPMA
    V, lf = 200, 16
    k = all_keys(V, 4)
    a = GPMA(V, dev(k[:5000]), leaf_size=lf, mirror=True, allocator=False)
    b = GPMA(V, dev(k[:5000]), leaf_size=lf, mirror=True)
    held0 = b.allocated_bytes
    for i in range(5000, 30000, 5000):
        for g in (a, b):
            g.insert(dev(k[i:i + 5000]))
            g.delete(dev(k[i - 5000:i - 2000]))
        assert np.array_equal(npu64(a.slots()), npu64(b.slots()))
    assert b.capacity > 2 * 8192 and b.allocated_bytes > held0
    assert a.allocated_bytes == b.allocated_bytes == b.allocator.held_bytes
    a.close()
    b.close()
