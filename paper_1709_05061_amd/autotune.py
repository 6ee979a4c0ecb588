"""Autotuner for the GPMA+ library: picks the leaf size for a workload by
timing the real update path (fused batching) on a sample of its batches.

The leaf length trades the cost of a leaf merge (16*lf bytes per merged leaf)
against how often merges climb above the leaves and how deep the leaf search
is; the best value depends on the graph's skew and on the batch sizes, so it
is measured rather than derived.  Results are cached in a JSON file keyed by
the workload's shape (vertices, initial edges, batch-size profile, mirror).
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence

import torch

from .gpma import GPMA

DEFAULT_CANDIDATES = (16, 32, 64, 128)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gpma_autotune.json")


def _key(V: int, n_init: int, sizes: Sequence[int], mirror: bool) -> str:
    h = hashlib.sha1(json.dumps([V, n_init, sorted(sizes), mirror]).encode()).hexdigest()[:16]
    return "V%d_n%d_%s" % (V, n_init, h)


def autotune_leaf_size(V: int, init_keys: torch.Tensor, ops: List[int], batches: List[torch.Tensor],
                       candidates: Sequence[int] = DEFAULT_CANDIDATES, mirror: bool = False,
                       cache_path: Optional[str] = DEFAULT_CACHE, warm: int = 2) -> Dict:
    """Time apply_batches(ops, batches) from the same initial graph for every
    candidate leaf size; returns {"leaf_size": best, "ms": {lf: ms}, "cached": bool}."""
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
    for lf in candidates:
        g = GPMA(V, init_keys, leaf_size=lf, mirror=mirror)
        # warm-up: the first batches capture the graphs of their size classes
        g.apply_batches(ops[:warm], batches[:warm])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.apply_batches(ops[warm:], batches[warm:])
        torch.cuda.synchronize()
        timings[lf] = 1e3 * (time.perf_counter() - t0)
        g.close()
        del g
    best = min(timings, key=timings.get)
    r = {"leaf_size": int(best), "ms": {str(k): v for k, v in timings.items()}, "cached": False}
    if cache_path:
        cache[key] = {"leaf_size": r["leaf_size"], "ms": r["ms"]}
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return r
