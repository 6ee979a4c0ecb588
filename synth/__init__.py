"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds no arithmetic of the method itself: only random draws, graph
generators and stream (sliding-window) layouts.

Every draw comes from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw i of stream `seed` is mix(seed + (i+1)*0x9E3779B97F4A7C15).
All arithmetic is on int64 tensors with wrap-around, so the same call gives
bit-identical results on the CPU and on a GPU device.

Workload shapes follow the paper's experiments (Section 6.1 "Datasets",
"Stream Setup"):
  * Erdos-Renyi random directed graphs (the "Random" dataset);
  * R-MAT graphs with a=0.57, b=0.19, c=0.19, d=0.05 (the Graph500 dataset);
  * random timestamps = a seeded random permutation of the edges; the window
    is a fixed-size prefix and slides by deleting its oldest edges and
    inserting the next ones.
"""
from __future__ import annotations

from typing import List, Tuple

import torch

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
GUARD_DST = 0xFFFFFFFF


def _s64(x: int) -> int:
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix64(counter: torch.Tensor, seed: int) -> torch.Tensor:
    """Output `counter` (0-based, int64 tensor) of the SplitMix64 stream whose
    state starts at `seed`; returns int64 bit patterns of the uint64 outputs."""
    z = counter.to(torch.int64) + 1
    z = z * _s64(_GAMMA) + _s64(seed)
    z = (z ^ _srl(z, 30)) * _s64(_M1)
    z = (z ^ _srl(z, 27)) * _s64(_M2)
    return z ^ _srl(z, 31)


def splitmix64_ref(seed: int, n: int):
    """The published sequential form, in Python integers (used by tests)."""
    x = seed & ((1 << 64) - 1)
    out = []
    for _ in range(n):
        x = (x + _GAMMA) & ((1 << 64) - 1)
        z = x
        z = ((z ^ (z >> 30)) * _M1) & ((1 << 64) - 1)
        z = ((z ^ (z >> 27)) * _M2) & ((1 << 64) - 1)
        out.append(z ^ (z >> 31))
    return out


def to_u64(t: torch.Tensor) -> int:
    return int(t) & ((1 << 64) - 1)


def edge_key(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    return (src.to(torch.int64) << 32) | dst.to(torch.int64)


def key_src(k: torch.Tensor) -> torch.Tensor:
    return _srl(k, 32)


def key_dst(k: torch.Tensor) -> torch.Tensor:
    return k & 0xFFFFFFFF


def unique_first(keys: torch.Tensor) -> torch.Tensor:
    """Distinct keys in order of first appearance."""
    if keys.numel() == 0:
        return keys
    sk, perm = torch.sort(keys, stable=True)
    first = torch.ones_like(sk, dtype=torch.bool)
    first[1:] = sk[1:] != sk[:-1]
    keep = torch.zeros_like(keys, dtype=torch.bool)
    keep[perm[first]] = True
    return keys[keep]


def shuffle(keys: torch.Tensor, seed: int) -> torch.Tensor:
    """Random timestamps: a seeded permutation (stable sort on random keys)."""
    r = splitmix64(torch.arange(keys.numel(), device=keys.device), seed)
    _, perm = torch.sort(r, stable=True)
    return keys[perm]


def uniform_below(counter: torch.Tensor, seed: int, n: int) -> torch.Tensor:
    """Integers in [0, n): the high 32 bits r of a draw, scaled to
    floor(r * n / 2^32) (0 <= n < 2^32).  The product is formed in two
    16-bit halves of n, so it stays inside int64 for every n."""
    if not 0 <= n < (1 << 32):
        raise ValueError("uniform_below needs 0 <= n < 2^32")
    r = _srl(splitmix64(counter, seed), 32)
    return (r * (n >> 16) + ((r * (n & 0xFFFF)) >> 16)) >> 16


# --------------------------------------------------------------------------
# graphs

def er_edges(V: int, m: int, seed: int, device="cpu", chunk: int = 1 << 22) -> torch.Tensor:
    """m distinct directed edges (u,v), u != v, uniform over V*(V-1) pairs, in
    draw order (which serves as their random timestamps).  This is G(n, m),
    the fixed-edge-count form of the paper's Erdos-Renyi "Random" graph."""
    assert m <= V * (V - 1)
    got = torch.empty(0, dtype=torch.int64, device=device)
    base = 0
    while got.numel() < m:
        n = max(chunk, 2 * (m - got.numel()))
        c = torch.arange(base, base + n, device=device, dtype=torch.int64)
        src = uniform_below(2 * c, seed, V)
        dst = uniform_below(2 * c + 1, seed, V)
        k = edge_key(src, dst)[src != dst]
        got = unique_first(torch.cat([got, k]))
        base += n
    return got[:m]


# integer quadrant thresholds on a 32-bit uniform: a, a+b, a+b+c of 2^32
def _rmat_thresholds(a: float, b: float, c: float):
    return (int(round(a * 2**32)), int(round((a + b) * 2**32)), int(round((a + b + c) * 2**32)))


def rmat_draws(scale: int, first: int, count: int, seed: int, a=0.57, b=0.19, c=0.19,
               device="cpu") -> torch.Tensor:
    """R-MAT draws number first..first+count-1 (Chakrabarti et al. 2004, the
    Graph500 generator's kernel): at each of `scale` bit levels one quadrant
    is picked with probabilities a, b, c, d=1-a-b-c; no noise, no vertex
    permutation.  Returns keys src<<32|dst (repeats and self-loops kept)."""
    ta, tb, tc = _rmat_thresholds(a, b, c)
    words = (scale + 1) // 2
    idx = torch.arange(first, first + count, device=device, dtype=torch.int64)
    src = torch.zeros(count, dtype=torch.int64, device=device)
    dst = torch.zeros(count, dtype=torch.int64, device=device)
    for w in range(words):
        r = splitmix64(idx * words + w, seed)
        for half in range(2):
            lvl = 2 * w + half
            if lvl >= scale:
                break
            u = _srl(r, 32) if half == 0 else (r & 0xFFFFFFFF)
            sb = (u >= tb).to(torch.int64)                        # quadrants c, d
            db = ((u >= ta) & (u < tb)) | (u >= tc)               # quadrants b, d
            bit = scale - 1 - lvl
            src |= sb << bit
            dst |= db.to(torch.int64) << bit
    return edge_key(src, dst)


def rmat_unique(scale: int, n_draws: int, seed: int, device="cpu", chunk: int = 1 << 24,
                **abc) -> torch.Tensor:
    """Distinct keys among the first n_draws R-MAT draws, sorted."""
    parts = []
    for f in range(0, n_draws, chunk):
        parts.append(torch.unique(rmat_draws(scale, f, min(chunk, n_draws - f), seed,
                                             device=device, **abc)))
    return torch.unique(torch.cat(parts))


# --------------------------------------------------------------------------
# sliding-window streams (Section 6.1 "Stream Setup")

class Stream:
    """An edge stream in timestamp order: the window initially holds
    `order[:window]`; slide t deletes order[t*b:(t+1)*b] (the oldest) and
    inserts order[window+t*b : window+(t+1)*b] (the next arrivals)."""

    def __init__(self, V: int, order: torch.Tensor, window: int):
        self.V = V
        self.order = order
        self.window = window

    def initial(self) -> torch.Tensor:
        return self.order[: self.window]

    def max_slides(self, b: int) -> int:
        return (self.order.numel() - self.window) // b

    def slide(self, t: int, b: int):
        dels = self.order[t * b:(t + 1) * b]
        ins = self.order[self.window + t * b: self.window + (t + 1) * b]
        return dels, ins

    def window_after(self, t: int, b: int) -> torch.Tensor:
        """Window content after slides 0..t-1 (unsorted)."""
        return self.order[t * b: self.window + t * b]


def er_stream(V: int, window: int, b: int, slides: int, seed: int, device="cpu") -> Stream:
    """The "Random" setup at a given size: distinct random edges in random
    timestamp order, a window of `window` edges and `slides` slides of b."""
    m = window + b * slides
    return Stream(V, er_edges(V, m, seed, device=device), window)


def rmat_stream(scale: int, edge_factor: int, seed: int, device="cpu") -> Stream:
    """Graph500-style setup: the distinct edges of edge_factor*2^scale R-MAT
    draws in random timestamp order; the first half is the initial window."""
    u = rmat_unique(scale, edge_factor << scale, seed, device=device)
    order = shuffle(u, seed ^ 0x5DEECE66D)
    return Stream(1 << scale, order, order.numel() // 2)


def rmat_full_stream(scale: int, edge_factor: int, extra_draws: int, seed: int,
                     device="cpu") -> Stream:
    """All distinct edges of edge_factor*2^scale draws form the initial window
    (in random timestamp order); arrivals are the distinct edges of the
    following `extra_draws` draws that are not already in the window, in draw
    order."""
    n = edge_factor << scale
    win = shuffle(rmat_unique(scale, n, seed, device=device), seed ^ 0x5DEECE66D)
    fresh = unique_first(rmat_draws(scale, n, extra_draws, seed, device=device))
    fresh = fresh[~torch.isin(fresh, win)]
    return Stream(1 << scale, torch.cat([win, fresh]), win.numel())


def explicit_deletion_slides(window: torch.Tensor, arrivals: torch.Tensor, b: int, slides: int,
                             seed: int) -> List[Tuple[torch.Tensor, torch.Tensor]]:
    """Graph stream with explicit deletions (the paper's extended experiment,
    Appendix "Graph Streams with Explicit Deletions"): each slide deletes b
    edges drawn at random from the current window (not the oldest) and
    inserts the next b arrivals.  Returns [(deletes, inserts)] per slide."""
    live = window.clone()
    out = []
    for t in range(slides):
        ins = arrivals[t * b:(t + 1) * b]
        ctr = torch.arange(2 * b, device=live.device, dtype=torch.int64) + (t << 32)
        idx = unique_first(uniform_below(ctr, seed, live.numel()))[:b]
        dels = live[idx]
        keep = torch.ones(live.numel(), dtype=torch.bool, device=live.device)
        keep[idx] = False
        live = torch.cat([live[keep], ins])
        out.append((dels, ins))
    return out


def sorted_stream(stream: "Stream") -> "Stream":
    """The same window, with the arrivals in ascending key order: every batch
    of inserts lands in one narrow key range, so merges climb the tree (the
    worst case of the PMA's amortized update cost, the lemma of Section 4.1)."""
    arr = stream.order[stream.window:]
    arr = torch.sort(arr).values
    return Stream(stream.V, torch.cat([stream.order[:stream.window], arr]), stream.window)


def uniform01(counter: torch.Tensor, seed: int) -> torch.Tensor:
    """Doubles in (0, 1) from the top 53 bits of a draw."""
    r = _srl(splitmix64(counter, seed), 11)
    return (r.to(torch.float64) + 0.5) / float(1 << 53)


def powerlaw_edges(V: int, m: int, seed: int, alpha: float = 2.1, device="cpu") -> torch.Tensor:
    """A social-network-shaped directed graph (Chung-Lu style): out-degrees
    follow a discrete power law with exponent `alpha` (Pareto weights,
    truncated at V, rescaled to about m edges in total); destinations are
    drawn with probability proportional to (rank+1)^(-1/(alpha-1)) over a
    seeded random ranking of the vertices.  Distinct edges without
    self-loops, in random order; topped up with further draws to m."""
    idx = torch.arange(V, device=device, dtype=torch.int64)
    w = uniform01(idx, seed) ** (-1.0 / (alpha - 1.0))
    w = torch.clamp(w, max=float(V))
    deg = torch.floor(w * (m * 1.15 / float(w.sum())) + uniform01(idx, seed + 1)).to(torch.int64)
    rank = torch.argsort(splitmix64(idx, seed + 2))
    zw = (rank.to(torch.float64) + 1.0) ** (-1.0 / (alpha - 1.0))
    cdf = torch.cumsum(zw, 0)
    cdf = cdf / cdf[-1]
    got = torch.empty(0, dtype=torch.int64, device=device)
    base = 0
    rnd = 0
    while got.numel() < m and rnd < 8:
        src = torch.repeat_interleave(idx, deg) if rnd == 0 else \
            uniform_below(torch.arange(base, base + 2 * (m - got.numel()), device=device), seed + 3, V)
        c = torch.arange(base, base + src.numel(), device=device, dtype=torch.int64)
        dst = torch.searchsorted(cdf, uniform01(c, seed + 4)).clamp(max=V - 1)
        k = edge_key(src, dst)[src != dst]
        k = k[torch.argsort(splitmix64(torch.arange(k.numel(), device=device), seed + 5 + rnd))]
        got = unique_first(torch.cat([got, k]))
        base += src.numel()
        rnd += 1
    return got[:m]


def poisson_times(n: int, rate: float, seed: int, device="cpu") -> torch.Tensor:
    """Arrival times (seconds, float64, ascending) of the first n events of a
    Poisson process with the given rate: cumulative exponential gaps."""
    u = uniform01(torch.arange(n, device=device), seed)
    return torch.cumsum(-torch.log(u) / rate, 0)


def loguniform_sizes(n: int, lo_log2: int, hi_log2: int, seed: int):
    """n batch sizes, log-uniform on [2^lo, 2^hi] (host integers)."""
    u = uniform01(torch.arange(n), seed)
    return [int(round(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * float(x)))) for x in u]


def random_batch(V: int, b: int, seed: int, device="cpu") -> torch.Tensor:
    """b uniform random edge keys (repeats and self-loops allowed)."""
    c = torch.arange(b, device=device, dtype=torch.int64)
    return edge_key(uniform_below(2 * c, seed, V), uniform_below(2 * c + 1, seed, V))
