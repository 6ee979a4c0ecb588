"""Autotuner for the GPMA+ library: picks the leaf size and the launch shape
for a workload by timing the real update path (fused batching) on a sample
of its batches.

Knobs:
  * leaf size -- trades the cost of a leaf merge (16*lf bytes per merged leaf)
    against how often merges climb above the leaves and how deep the leaf
    search is;
  * sort tile -- keys per workgroup tile of the batch radix sort (512, 1024
    or 2048): more, smaller tiles spread a small batch over more compute
    units but make every workgroup derive more digit offsets;
  * enqueue mode -- replay a captured HIP graph per batch, or enqueue the
    same kernels directly (the device-side control is identical; the cost of
    launching a graph versus its kernels depends on the runtime);
  * fused levels -- how many tree levels above the leaves each batch runs on
    the device: every covered level costs a few launches even when nothing
    reaches it, and an uncovered level that is reached costs a host round
    trip.
The best point depends on the graph's skew, the batch sizes and the runtime,
so it is measured rather than derived.  Results are cached in a JSON file
keyed by the workload's shape (vertices, initial edges, batch-size profile,
mirror).
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from typing import Dict, List, Optional, Sequence

import torch

from .gpma import GPMA

DEFAULT_LEAF_SIZES = (16, 32, 64, 128)
DEFAULT_SORT_TILES = (512, 1024, 2048)
DEFAULT_MODES = (False, True)   # fused_direct
DEFAULT_LEVELS = (0, 1, 2)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gpma_autotune.json")


def _key(V: int, n_init: int, sizes: Sequence[int], mirror: bool) -> str:
    h = hashlib.sha1(json.dumps([V, n_init, sorted(sizes), mirror]).encode()).hexdigest()[:16]
    return "V%d_n%d_%s" % (V, n_init, h)


def _name(lf: int, tile: int, direct: bool, levels: int) -> str:
    return "lf%d_tile%d_%s_lv%d" % (lf, tile, "direct" if direct else "graph", levels)


def autotune(V: int, init_keys: torch.Tensor, ops: List[int], batches: List[torch.Tensor],
             leaf_sizes: Sequence[int] = DEFAULT_LEAF_SIZES, sort_tiles: Sequence[int] = DEFAULT_SORT_TILES,
             modes: Sequence[bool] = DEFAULT_MODES, levels: Sequence[int] = DEFAULT_LEVELS,
             mirror: bool = False, learned: bool = False, cache_path: Optional[str] = DEFAULT_CACHE,
             warm: int = 2) -> Dict:
    """Time apply_batches(ops, batches) from the same initial graph for every
    (leaf size, sort tile, enqueue mode, fused levels); returns {"leaf_size",
    "sort_tile", "fused_direct", "fused_levels", "ms": {name: ms}, "cached"}."""
    sizes = [int(b.numel()) for b in batches]
    key = _key(V, int(init_keys.numel()), sizes, mirror)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            r = dict(cache[key])
            r["cached"] = True
            return r
    timings = {}
    best = None
    for lf, tile, direct, lv in itertools.product(leaf_sizes, sort_tiles, modes, levels):
        g = GPMA(V, init_keys, leaf_size=lf, mirror=mirror, learned=learned, fused_direct=direct,
                 sort_tile=tile, fused_levels=lv)
        # warm-up: the first batches capture the graphs of their size classes
        g.apply_batches(ops[:warm], batches[:warm])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.apply_batches(ops[warm:], batches[warm:])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        timings[_name(lf, tile, direct, lv)] = ms
        if best is None or ms < best[0]:
            best = (ms, lf, tile, direct, lv)
        g.close()
        del g
    r = {"leaf_size": int(best[1]), "sort_tile": int(best[2]), "fused_direct": bool(best[3]),
         "fused_levels": int(best[4]), "ms": timings, "cached": False}
    if cache_path:
        cache[key] = {k: v for k, v in r.items() if k != "cached"}
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return r


def autotune_leaf_size(V: int, init_keys: torch.Tensor, ops: List[int], batches: List[torch.Tensor],
                       candidates: Sequence[int] = DEFAULT_LEAF_SIZES, mirror: bool = False,
                       cache_path: Optional[str] = DEFAULT_CACHE, warm: int = 2) -> Dict:
    """Leaf size only (graph replay, default sort tile)."""
    return autotune(V, init_keys, ops, batches, leaf_sizes=candidates, sort_tiles=(1024,), modes=(False,),
                    levels=(1,), mirror=mirror, cache_path=cache_path, warm=warm)
