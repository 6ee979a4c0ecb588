"""The seeded input generators that the oracle and the GPU path share: each
is checked against its published definition or the distribution it claims,
so that a mistake in a recipe cannot hide behind both sides agreeing."""
import math

import numpy as np
import torch

import synth

U64 = (1 << 64) - 1


def u64(t: torch.Tensor):
    return [int(x) & U64 for x in t]


def test_splitmix64_published_outputs_and_counter_form():
    # the first outputs of SplitMix64 from state 0 (Steele, Lea, Flood 2014;
    # the values every reference implementation prints for seed 0)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert synth.splitmix64_ref(0, 3) == want
    assert u64(synth.splitmix64(torch.arange(3), 0)) == want
    # the counter form equals the sequential stream for any seed and counter
    for seed in (1, 12345, (1 << 63) + 7, U64):
        ref = synth.splitmix64_ref(seed, 300)
        assert u64(synth.splitmix64(torch.arange(300), seed)) == ref
        sel = torch.tensor([0, 17, 299])
        assert u64(synth.splitmix64(sel, seed)) == [ref[i] for i in sel.tolist()]


def test_uniform_below_and_uniform01():
    n = 7
    r = synth.uniform_below(torch.arange(70000), 3, n)
    assert int(r.min()) == 0 and int(r.max()) == n - 1
    counts = torch.bincount(r, minlength=n).tolist()
    assert all(abs(c - 10000) < 300 for c in counts), counts
    # floor(r * n / 2^32) of the draw's high 32 bits r, for n up to 2^32 - 1
    # (the int64 product r * n overflows from n = 2^31 on)
    c = torch.arange(3000)
    hi32 = [x >> 32 for x in u64(synth.splitmix64(c, 4))]
    for n in (1, 1000, (1 << 31) - 1, 1 << 31, 3_000_000_000, (1 << 32) - 1):
        assert synth.uniform_below(c, 4, n).tolist() == [(x * n) >> 32 for x in hi32], n
    u = synth.uniform01(torch.arange(100000), 5)
    assert float(u.min()) > 0.0 and float(u.max()) < 1.0
    assert abs(float(u.mean()) - 0.5) < 0.005


def test_rmat_quadrant_probabilities_at_every_level():
    # each bit level picks quadrant a (0,0), b (0,1), c (1,0), d (1,1)
    # independently with the stated probabilities
    scale, n = 8, 1 << 17
    a, b, c = 0.57, 0.19, 0.19
    k = synth.rmat_draws(scale, 0, n, 11)
    src, dst = synth.key_src(k), synth.key_dst(k)
    assert int(src.max()) < (1 << scale) and int(dst.max()) < (1 << scale)
    for bit in range(scale):
        s = (src >> bit) & 1
        d = (dst >> bit) & 1
        got = [float(((s == x) & (d == y)).double().mean()) for x, y in ((0, 0), (0, 1), (1, 0), (1, 1))]
        for g, p in zip(got, (a, b, c, 1 - a - b - c)):
            assert abs(g - p) < 0.006, (bit, got)
    # with b != c the quadrants keep their places: b sets the destination
    # bit only, c the source bit only
    k2 = synth.rmat_draws(4, 0, 1 << 16, 13, a=0.5, b=0.3, c=0.1)
    s2, d2 = synth.key_src(k2) & 1, synth.key_dst(k2) & 1
    assert abs(float(((s2 == 0) & (d2 == 1)).double().mean()) - 0.3) < 0.01
    assert abs(float(((s2 == 1) & (d2 == 0)).double().mean()) - 0.1) < 0.01
    # counter-based: any split of the draw range gives the same draws
    whole = synth.rmat_draws(scale, 100, 1000, 11)
    parts = torch.cat([synth.rmat_draws(scale, 100, 400, 11), synth.rmat_draws(scale, 500, 600, 11)])
    assert torch.equal(whole, parts)
    # a = b = c = 1/4 is the uniform distribution over all V*V pairs
    uni = synth.rmat_draws(4, 0, 1 << 16, 12, a=0.25, b=0.25, c=0.25)
    cnt = torch.bincount(synth.key_src(uni) * 16 + synth.key_dst(uni), minlength=256).double()
    assert float(((cnt - 256.0) ** 2 / 256.0).sum()) < 340.0   # chi-square, 255 degrees of freedom


def test_rmat_full_stream_window_and_arrivals():
    scale, ef, extra = 10, 8, 1 << 13
    st = synth.rmat_full_stream(scale, ef, extra, 21)
    win = st.initial()
    arr = st.order[st.window:]
    assert st.V == 1 << scale
    assert torch.equal(torch.sort(win).values, synth.rmat_unique(scale, ef << scale, 21))
    assert torch.unique(arr).numel() == arr.numel()
    assert not bool(torch.isin(arr, win).any())
    # arrivals are the later draws' first appearances, in draw order
    later = synth.unique_first(synth.rmat_draws(scale, ef << scale, extra, 21))
    assert torch.equal(arr, later[~torch.isin(later, win)])
    # slide t deletes the oldest b edges and inserts the next b arrivals
    b = 100
    d, i = st.slide(2, b)
    assert torch.equal(d, win[2 * b:3 * b]) and torch.equal(i, arr[2 * b:3 * b])
    assert torch.equal(st.window_after(2, b), torch.cat([win[2 * b:], arr[:2 * b]]))


def test_er_and_powerlaw_edges_are_distinct_without_self_loops():
    V, m = 1 << 12, 1 << 15
    for e in (synth.er_edges(V, m, 31), synth.powerlaw_edges(V, m, 32)):
        assert e.numel() == m and torch.unique(e).numel() == m
        s, d = synth.key_src(e), synth.key_dst(e)
        assert not bool((s == d).any())
        assert int(s.max()) < V and int(d.max()) < V
    # the power-law graph is heavy-tailed on both sides; ER's degrees are
    # near their mean (binomial, mean 8)
    pl = synth.powerlaw_edges(V, m, 32)
    out_pl = torch.bincount(synth.key_src(pl), minlength=V)
    in_pl = torch.bincount(synth.key_dst(pl), minlength=V)
    out_er = torch.bincount(synth.key_src(synth.er_edges(V, m, 31)), minlength=V)
    mean = m / V
    assert int(out_pl.max()) > 20 * mean and int(in_pl.max()) > 20 * mean
    assert int(out_er.max()) < 4 * mean


def test_poisson_times_and_loguniform_sizes():
    rate, n = 2.5e4, 100000
    t = synth.poisson_times(n, rate, 41)
    gaps = torch.diff(t)
    assert bool((gaps > 0).all()) and float(t[0]) > 0
    mean = float(t[-1]) / n
    assert abs(mean * rate - 1.0) < 0.02
    cv = float(gaps.std()) / float(gaps.mean())
    assert abs(cv - 1.0) < 0.03   # exponential gaps: standard deviation = mean
    sizes = synth.loguniform_sizes(4000, 6, 18, 42)
    assert min(sizes) >= 1 << 6 and max(sizes) <= 1 << 18
    lg = np.log2(np.array(sizes, dtype=np.float64))
    assert abs(lg.mean() - 12.0) < 0.15
    assert abs(lg.std() - 12.0 / math.sqrt(12.0)) < 0.15   # uniform on [6, 18]
