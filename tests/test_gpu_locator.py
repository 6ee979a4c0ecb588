"""Learned segment locator: the row span from the CSR offsets plus the MFMA
model of the destination's place in it, corrected by a bounded search,
returns the binary-search leaf for every key and keeps the layout
slot-identical to the oracle; its window stays far below the array and
fallbacks are rare."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def npu64(t):
    return t.cpu().numpy().view(np.uint64)


def dev(keys):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).view(np.int64)).cuda()


@pytest.mark.parametrize("kind", ["er", "rmat"])
def test_learned_locate_equals_binary_search(kind):
    from paper_1709_05061_amd import GPMA
    if kind == "er":
        V = 1 << 14
        e = synth.er_edges(V, 1 << 17, seed=1)
    else:
        V = 1 << 15
        e = synth.rmat_unique(15, 16 << 15, seed=2)
    learned = GPMA(V, e.cuda(), leaf_size=32, learned=True)
    plain = GPMA(V, e.cuda(), leaf_size=32)
    probe = torch.cat([synth.random_batch(V, 50000, 3).cuda(), e[:20000].cuda(),
                       torch.tensor([0, (V - 1) << 32 | (V - 1)], device="cuda")])
    a = learned.locate(probe).cpu().numpy()
    b = plain.locate(probe).cpu().numpy()
    assert np.array_equal(a, b)
    info = learned.locator_info()
    print(kind, info, flush=True)
    if kind == "er":
        assert info["eps"] <= 64           # the model is accurate on a uniform CDF
        assert info["misses"] * 100 <= info["lookups"]
    else:
        assert info["eps"] < learned.capacity // 32   # a real window, not the whole array
        assert info["misses"] * 20 <= info["lookups"]
    learned.close()
    plain.close()


@pytest.mark.parametrize("mirror", [False, True])
def test_learned_locator_keeps_layout(mirror):
    """Sliding window with the learned locator (refits after resizes and
    when lookups fall back): slot-identical to the oracle after every batch,
    plain and fused."""
    from paper_1709_05061_amd import GPMA
    V, lf = 1 << 12, 16
    st = synth.er_stream(V, 1 << 15, 1 << 9, 12, seed=7)
    init = npu64(st.initial())
    g = GPMA(V, dev(init), leaf_size=lf, learned=True, mirror=mirror)
    f = GPMA(V, dev(init), leaf_size=lf, learned=True, mirror=mirror)
    ref = O.OraclePMA(V, init, lf)
    for t in range(12):
        d, i = st.slide(t, 1 << 9)
        g.delete(d.cuda())
        g.insert(i.cuda())
        f.apply_batches([1, 0], [d.cuda(), i.cuda()])
        ref.delete(npu64(d))
        ref.insert(npu64(i))
        assert np.array_equal(npu64(g.slots()), ref.slots()), t
        assert np.array_equal(npu64(f.slots()), ref.slots()), t
    big = npu64(synth.random_batch(V, 40000, 8))   # forces a resize, then a refit
    g.insert(dev(big))
    ref.insert(big)
    assert np.array_equal(npu64(g.slots()), ref.slots())
    assert g.locator_info()["fits"] >= 2
    g.close()
    f.close()
