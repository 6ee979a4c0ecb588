"""Benchmark of the GPMA+ hot path on one MI355X.

Workload (the headline configuration): an R-MAT graph (a=.57, b=c=.19,
d=.05), scale 24, edge factor 16: all distinct edges of 2^28 draws form the
initial window (~2.4e8 edges, a 2^29-slot = 4 GiB PMA).  One step slides the
window once: delete the 2^16 oldest edges, insert 2^16 fresh ones, then run
the analytics of the stream (PageRank 10 iterations warm-started from the
previous step, BFS from a random vertex, connected components).  By default
the handle keeps the dst-major mirror (both arrays take every batch, and
PageRank pulls over the mirror); --no-mirror pushes with fp64 atomics.

value     = edge updates applied per second of update time (delete + insert
            phases of the timed steps, HIP events on the update stream)
roofline  = the dominant kernel by time (PageRank's SpMV), algorithmic bytes
            per launch / its mean launch time from HIP events
cpu_baseline = the CPU oracle (single thread) on a bounded sample: an R-MAT
            scale-20 window with the same 2^16-edge slides.

Inputs are generated on the device before the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge updates/sec at batch 2^16 (R-MAT s24) + SpMV GB/s; p99 stream latency"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pctl(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def cpu_baseline(batch: int, slides: int, scale: int = 20):
    """Time the oracle (as it stands) on one host core over a bounded sample."""
    import numpy as np
    import torch

    import oracle as O
    import synth
    dev = "cuda" if torch.cuda.is_available() else "cpu"
    st = synth.rmat_stream(scale, 16, seed=1, device=dev)
    order = st.order.cpu().numpy().view(np.uint64)
    p = O.OraclePMA(st.V, order[: st.window], 32)
    t0 = time.perf_counter()
    applied = 0
    for t in range(slides):
        p.delete(order[t * batch:(t + 1) * batch])
        applied += p.last_applied()
        p.insert(order[st.window + t * batch: st.window + (t + 1) * batch])
        applied += p.last_applied()
    dt = time.perf_counter() - t0
    edges = O.edge_keys(p.slots())
    t1 = time.perf_counter()
    O.pagerank(st.V, edges, iters=10)
    dpr = time.perf_counter() - t1
    spmv_bytes = 10 * (8.0 * (edges.size + st.V) + 16.0 * st.V)
    return {
        "value": applied / dt,
        "unit": "edge updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "R-MAT scale %d edge factor 16 window (%d edges), %d slides of %d deletes + %d "
                  "inserts, single thread" % (scale, st.window, slides, batch, batch),
        "seconds": dt,
        "pagerank_spmv_GBps": spmv_bytes / dpr / 1e9,
        "pagerank_seconds": dpr,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--batch", type=int, default=1 << 16)
    ap.add_argument("--leaf-size", type=int, default=0)
    ap.add_argument("--pr-iters", type=int, default=10)
    ap.add_argument("--no-analytics", action="store_true")
    ap.add_argument("--no-mirror", action="store_true",
                    help="no dst-major mirror: PageRank pushes with fp64 atomics")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slides", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the PMA would shard by vertex range; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd import gpma as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    b = args.batch
    need = (args.warmup + args.steps) * b
    t0 = time.time()
    extra = max(4 * need, 1 << 22)
    while True:
        st = synth.rmat_full_stream(args.scale, args.edge_factor, extra, args.seed, device="cuda")
        if st.order.numel() - st.window >= need:
            break
        extra *= 2
    V = st.V
    torch.cuda.synchronize()
    log("generated R-MAT s%d: window %d edges, %d fresh arrivals in %.1fs"
        % (args.scale, st.window, st.order.numel() - st.window, time.time() - t0))
    t0 = time.time()
    g = GPMA(V, st.initial(), leaf_size=args.leaf_size, mirror=not args.no_mirror)
    torch.cuda.synchronize()
    log("created PMA: %d edges, capacity %d slots, leaf %d in %.1fs"
        % (g.num_edges, g.capacity, g.leaf_size, time.time() - t0))

    # BFS sources: vertices with out-edges, drawn with the seeded generator
    deg = g.degrees()
    cand = torch.nonzero(deg > 0).flatten()
    pick = synth.uniform_below(torch.arange(args.warmup + args.steps, device="cuda"), args.seed + 7,
                               cand.numel())
    sources = cand[pick].tolist()

    stream = torch.cuda.current_stream()
    x = torch.full((V,), 1.0 / V, dtype=torch.float32, device="cuda")

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def step(t, timed):
        d, i = st.slide(t, b)
        e0 = ev()
        sd = g.delete(d, stats=True)
        si = g.insert(i, stats=True)
        e1 = ev()
        marks = [e0, e1]
        if not args.no_analytics:
            g.pagerank(init=x, iters=args.pr_iters, out=x)
            marks.append(ev())
            g.bfs(sources[t])
            marks.append(ev())
            g.cc()
            marks.append(ev())
        return sd, si, marks

    for t in range(args.warmup):
        step(t, False)
    torch.cuda.synchronize()
    g.profile_reset()
    g.profile(True)
    recs = []
    applied = 0
    resized = 0
    torch.cuda.synchronize()
    tw0 = time.perf_counter()
    for t in range(args.warmup, args.warmup + args.steps):
        sd, si, marks = step(t, True)
        applied += sd.applied + si.applied
        resized += int(sd.resized) + int(si.resized)
        recs.append(marks)
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw0
    g.profile(False)

    upd_ms = [m[0].elapsed_time(m[1]) for m in recs]
    phases = {"update": sum(upd_ms) / len(recs)}
    if not args.no_analytics:
        phases["pagerank"] = sum(m[1].elapsed_time(m[2]) for m in recs) / len(recs)
        phases["bfs"] = sum(m[2].elapsed_time(m[3]) for m in recs) / len(recs)
        phases["cc"] = sum(m[3].elapsed_time(m[4]) for m in recs) / len(recs)
    updates_per_s = applied / (sum(upd_ms) / 1e3)

    kernels = {}
    for kid, name in enumerate(G.KERNEL_NAMES):
        ms, n, by = g.profile_read(kid)
        if n:
            kernels[name] = {"launches": n, "mean_us": 1e3 * ms / n, "total_ms": ms,
                             "GBps": (by / (ms / 1e3) / 1e9) if by and ms else None}
    dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
    dom_name, dom_k = dom
    achieved = dom_k["GBps"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBPS) if achieved else None, "traffic": None,
                "kernel": dom_name}
    spmv = kernels.get("spmv")
    out = {
        "metric": METRIC,
        "value": updates_per_s,
        "unit": "edge updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "R-MAT scale %d edge factor %d sliding window; per step %d deletes + "
                               "%d inserts, PageRank %d iters (warm start), BFS, CC"
                               % (args.scale, args.edge_factor, b, b, args.pr_iters),
                   "scale": args.scale, "edge_factor": args.edge_factor, "batch": b,
                   "window_edges": int(st.window), "capacity": g.capacity, "leaf_size": g.leaf_size,
                   "mirror": not args.no_mirror},
        "phases_ms": phases,
        "update_ms_p50": pctl(upd_ms, 50),
        "update_ms_p99": pctl(upd_ms, 99),
        "applied_per_step": applied / args.steps,
        "resizes": resized,
        "spmv_GBps": spmv["GBps"] if spmv else None,
        "spmv_frac": (spmv["GBps"] / HBM_PEAK_GBPS) if spmv and spmv["GBps"] else None,
        "kernels": kernels,
        "roofline": roofline,
    }
    g.close()
    del st
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_slides)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
