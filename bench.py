"""Benchmark of the GPMA+ hot path on one MI355X.

Workload (the headline configuration): an R-MAT graph (a=.57, b=c=.19,
d=.05), scale 24, edge factor 16: all distinct edges of 2^28 draws form the
initial window (~2.4e8 edges, a 2^29-slot = 4 GiB PMA).  One step slides the
window once: delete the 2^16 oldest edges, insert 2^16 fresh ones, then run
the analytics of the stream (PageRank 10 iterations warm-started from the
previous step, BFS from a random vertex, connected components).  By default
the handle keeps the dst-major mirror (both arrays take every batch; it
serves bottom-up BFS and the CC sampling; PageRank uses destination bins
either way).

Beside the headline: the other update path (plain or fused) on the same
slides, the same configuration with lazy deletion, and two comparators on
the first slides: a CSR rebuilt per batch and the lock-based GPMA (against
GPMA+ on the same handle configuration, both with lazy deletion).

value     = edge updates applied per second of update time (delete + insert
            phases of the timed steps, HIP events on the update stream)
roofline  = the dominant kernel by time (PageRank's SpMV), algorithmic bytes
            per launch / its mean launch time from HIP events
cpu_baseline = the CPU oracle (single thread) on the headline inputs: the
            first slides through the sequential layout oracle (and the
            sorted-vector set), with the host's CPU model and core count.

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


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summaries
    under profiles/ (FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel of
    known size), or None when there is none or its kernel source has changed
    since the counters were taken."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    for path in sorted(glob.glob(os.path.join(here, "profiles", "*_traffic.md"))):
        fields = {}
        with open(path) as f:
            for line in f:
                k, sep, v = line.partition(":")
                if sep and k.strip() in ("traffic_kernel", "traffic_bytes_per_launch", "source", "source_sha256"):
                    fields[k.strip()] = v.strip()
        if fields.get("traffic_kernel") != kernel or "source" not in fields:
            continue
        src = os.path.join(here, fields["source"])
        if not os.path.exists(src):
            continue
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != fields.get("source_sha256"):
                continue
        return float(fields["traffic_bytes_per_launch"])
    return None


def host_cpu() -> dict:
    """The host's CPU model and core counts (what the CPU figures ran on)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(st, batch: int, layout_slides: int, set_slides: int, pr: bool = True):
    """Time the oracle (as it stands, one thread) on the headline inputs: the
    same R-MAT window and the same slides the GPU path applies.  The layout
    oracle (the sequential GPMA+) does work linear in the capacity per batch,
    seconds at this size, so it takes `layout_slides` slides; the semantic
    sorted-vector set takes `set_slides`.  PageRank: one fp64 10-step call on
    the oracle's edge set."""
    import numpy as np
    import torch

    import oracle as O
    win = torch.sort(st.order[: st.window])[0]      # a set: sorted only to spare the oracle's sort
    init = win.cpu().numpy().view(np.uint64)
    del win

    def slide(t):
        d, i = st.slide(t, batch)
        return d.cpu().numpy().view(np.uint64), i.cpu().numpy().view(np.uint64)

    slides = {t: slide(t) for t in range(max(layout_slides, set_slides))}
    out = {"unit": "edge updates/s", "cores": 1, "kind": "oracle", "host": host_cpu()}
    p = O.OraclePMA(st.V, init, 32)
    t0 = time.perf_counter()
    applied = 0
    for t in range(layout_slides):
        d, i = slides[t]
        p.delete(d)
        applied += p.last_applied()
        p.insert(i)
        applied += p.last_applied()
    dt = time.perf_counter() - t0
    out["value"] = applied / dt
    out["seconds"] = dt
    out["sample"] = ("the headline inputs (R-MAT scale %d window of %d edges, %d-slot array, leaf 32): "
                     "%d slides of %d deletes + %d inserts through the sequential layout oracle, "
                     "single thread" % (int(np.log2(st.V)), st.window, p.capacity, layout_slides, batch, batch))
    edges = O.edge_keys(p.slots())
    del p
    s = O.OracleSet(init)
    t0 = time.perf_counter()
    n = 0
    for t in range(set_slides):
        d, i = slides[t]
        n += s.delete(d) + s.insert(i)
    ds = time.perf_counter() - t0
    out["semantic_set"] = {"value": n / ds, "seconds": ds, "slides": set_slides,
                           "what": "sorted unique vector, each batch merged in or out (one thread)"}
    del s
    if pr:
        t1 = time.perf_counter()
        O.pagerank(st.V, edges, iters=10)
        dpr = time.perf_counter() - t1
        out["pagerank_seconds"] = dpr
        out["pagerank_spmv_GBps"] = 10 * (8.0 * (edges.size + st.V) + 28.0 * st.V) / dpr / 1e9
    return out


def sweep_slides(z: int) -> int:
    """Slides per batch size in the latency sweep (one of them a warm-up)."""
    return 11 if z <= (1 << 16) else (5 if z <= (1 << 18) else 4)


def spmv_forms_section(args, g, st, V, kernels):
    """PageRank's SpMV in both binned forms on the headline graph: the
    headline handle's own form (timed in the steps) and the other one on a
    handle of the initial window (no mirror).  Per form: mean SpMV time over
    the iterations of two 10-iteration calls, algorithmic GB/s, and the
    whole call's time (the per-call binning included)."""
    import torch

    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd import gpma as G
    own = "binned_gather" if args.spmv in ("auto", "binned_gather") else args.spmv
    out = {own: {"spmv_mean_us": kernels["spmv"]["mean_us"], "GBps": kernels["spmv"]["GBps"],
                 "source": "headline steps"}} if "spmv" in kernels else {}
    for form in ("binned", "binned_gather"):
        if form in out:
            continue
        h = GPMA(V, st.initial(), spmv=form)
        x = torch.full((V,), 1.0 / V, dtype=torch.float32, device="cuda")
        h.pagerank(init=x, iters=args.pr_iters, out=x)
        torch.cuda.synchronize()
        h.profile_reset()
        h.profile(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(2):
            h.pagerank(init=x, iters=args.pr_iters, out=x)
        t1.record()
        torch.cuda.synchronize()
        h.profile(False)
        ms, n, by = h.profile_read(G.K_SPMV)
        out[form] = {"spmv_mean_us": 1e3 * ms / n, "GBps": by / (ms / 1e3) / 1e9,
                     "pagerank_call_ms": t0.elapsed_time(t1) / 2, "source": "initial window, no mirror"}
        log("SpMV form %s: %s" % (form, out[form]))
        h.close()
        del h
        torch.cuda.empty_cache()
    return out


def resize_section(args):
    """A root doubling at the headline size (Algorithm GPMA+, the root's
    resize): the scale-24 window in a handle whose upper bound is the same at
    every level (tau about .53, rho_root .25), which puts its 2.8e8 entries just
    under the bound of 2^29 slots, then one insert batch of 2^22 fresh edges:
    the leaves and every segment above them fail their bound, so the batch
    climbs to the root, which cannot take it either: every entry is gathered,
    merged with the batch and re-dispatched over 2^30 slots (4 -> 8 GiB).  Reported: the batch's time, the capacities and
    its bytes (read 8 B a slot of the old array, write 8 B a slot of the new
    one, the merge's read and write of every entry)."""
    import torch

    import synth
    from paper_1709_05061_amd import GPMA
    st = synth.rmat_full_stream(24, 16, 1 << 23, args.seed + 60, device="cuda")
    # the root bound just above the window's entries plus half the batch
    n_entries = st.window + st.V
    tau_pm = -(-1000 * (n_entries + (1 << 21)) // (1 << 29))
    g = GPMA(st.V, st.initial(), tau_leaf=tau_pm, tau_root=tau_pm, rho_root=250)
    cap0, n0 = g.capacity, g.num_edges + st.V
    batch = st.order[st.window: st.window + (1 << 22)]
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s = g.insert(batch, stats=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    n1 = g.num_edges + st.V
    by = 8.0 * cap0 + 8.0 * g.capacity + 16.0 * n1 + 8.0 * batch.numel()
    out = {"workload": "R-MAT scale 24 window (%d edges) under tau .%03d at every level; one insert batch of %d edges"
                       % (st.window, tau_pm, batch.numel()),
           "capacity_before": cap0, "capacity_after": g.capacity, "resized": bool(s.resized),
           "entries_before": n0, "entries_after": n1, "applied": s.applied, "ms": ms,
           "bytes": by, "GBps": by / (ms / 1e3) / 1e9, "frac": by / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS}
    g.close()
    return out


def rmat20_section(args):
    """R-MAT scale 20 (window = the first half of the distinct edges): per
    batch size 2^10..2^20, 4 slides (fused, mirror, learned locator), each
    followed by BFS from 8 sources with out-edges, CC and 10-step PageRank."""
    import torch

    import synth
    from paper_1709_05061_amd import GPMA
    st = synth.rmat_stream(20, 16, args.seed + 70, device="cuda")
    g = GPMA(st.V, st.initial(), mirror=True, learned=True)
    deg = g.degrees()
    cand = torch.nonzero(deg > 0).flatten()
    srcs = cand[synth.uniform_below(torch.arange(8, device="cuda"), args.seed + 71, cand.numel())].tolist()
    out = {"workload": "R-MAT scale 20 edge factor 16, window %d edges; 4 slides per batch size, each "
                       "followed by BFS from 8 sources, CC and PageRank(10)" % st.window, "sizes": [],
           "update_ms": [], "updates_per_s": [], "bfs8_ms": [], "cc_ms": [], "pagerank_ms": []}
    t0 = 0
    x = torch.full((st.V,), 1.0 / st.V, dtype=torch.float32, device="cuda")
    for lb in range(10, 21, 2):
        z = 1 << lb
        rec = []
        for j in range(5):
            d, i = st.order[t0:t0 + z], st.order[st.window + t0: st.window + t0 + z]
            t0 += z
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            ev[0].record()
            a = g.apply_batches([1, 0], [d, i]).applied
            ev[1].record()
            for src in srcs:
                g.bfs(src)
            ev[2].record()
            g.cc()
            ev[3].record()
            g.pagerank(init=x, iters=10, out=x)
            ev[4].record()
            torch.cuda.synchronize()
            if j:   # the first slide of a size captures its graphs
                rec.append([a] + [ev[k].elapsed_time(ev[k + 1]) for k in range(4)])
        n = len(rec)
        out["sizes"].append(z)
        out["update_ms"].append(sum(r[1] for r in rec) / n)
        out["updates_per_s"].append(sum(r[0] for r in rec) / (sum(r[1] for r in rec) / 1e3))
        out["bfs8_ms"].append(sum(r[2] for r in rec) / n)
        out["cc_ms"].append(sum(r[3] for r in rec) / n)
        out["pagerank_ms"].append(sum(r[4] for r in rec) / n)
        log("R-MAT 20 b=%d: update %.3f ms, BFS x8 %.2f ms, CC %.2f ms, PageRank %.2f ms"
            % (z, out["update_ms"][-1], out["bfs8_ms"][-1], out["cc_ms"][-1], out["pagerank_ms"][-1]))
    g.close()
    return out


def uneven_section(args):
    """The fused-batching workload: a power-law social graph (1.6M vertices,
    30M edges, out-degree exponent 2.1), window = first half, then `n` slides
    of uneven size (log-uniform 2^6..2^18 each way), leaf size autotuned;
    fused vs plain update throughput at identical output."""
    import torch

    import synth
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd.autotune import autotune
    V, m = 1_600_000, 30_000_000
    e = synth.powerlaw_edges(V, m, seed=args.seed + 20, device="cuda")
    st = synth.Stream(V, e, e.numel() // 2)
    sizes = synth.loguniform_sizes(args.uneven_slides, 6, 18, args.seed + 21)
    ops, bs, pos = [], [], 0
    for b in sizes:
        ops += [1, 0]
        bs += [st.order[pos:pos + b], st.order[st.window + pos: st.window + pos + b]]
        pos += b
    tune = autotune(V, st.initial(), ops[:64], bs[:64], leaf_sizes=(16, 32, 64), sort_tiles=(512, 1024),
                    mirror=False, cache_path=None)
    lf = tune["leaf_size"]
    plain = GPMA(V, st.initial(), leaf_size=lf)
    fused = GPMA(V, st.initial(), leaf_size=lf, fused_direct=tune["fused_direct"], sort_tile=tune["sort_tile"],
                 fused_levels=tune["fused_levels"])
    fused.apply_batches(ops[:2], bs[:2])          # captures the first graphs
    plain.delete(bs[0])
    plain.insert(bs[1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for o, b in zip(ops[2:], bs[2:]):
        (plain.delete if o else plain.insert)(b)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    sf = fused.apply_batches(ops[2:], bs[2:])
    torch.cuda.synchronize()
    t_fused = time.perf_counter() - t0
    same = bool(torch.equal(plain.slots(), fused.slots()))
    n_upd = sum(int(b.numel()) for b in bs[2:])
    out = {"workload": "power-law graph V=1.6M, 30M edges, out-degree exponent 2.1, window 15M; "
                       "%d slides of log-uniform 2^6..2^18 deletes + inserts" % (len(sizes) - 1),
           "leaf_size": lf, "sort_tile": tune["sort_tile"], "fused_direct": tune["fused_direct"],
           "fused_levels": tune["fused_levels"],
           "autotune_ms": tune["ms"], "updates": n_upd,
           "plain_updates_per_s": n_upd / t_plain, "fused_updates_per_s": n_upd / t_fused,
           "fused_speedup": t_plain / t_fused, "identical_output": same, "applied": sf.applied}
    plain.close()
    fused.close()
    return out


def workloads_section(args):
    """The paper's other stream shapes at R-MAT scale 22, b = 2^16: explicit
    random deletions (each slide deletes random window edges instead of the
    oldest), a sorted arrival stream (every insert batch in one narrow key
    range), and window expiry with lazy deletion (deletes mark their entries
    in place) beside the same slides with merged deletions.  Plain and fused
    update throughput at identical output."""
    import torch

    import synth
    from paper_1709_05061_amd import GPMA
    b, slides = 1 << 16, 16
    st = synth.rmat_stream(22, 16, args.seed + 40, device="cuda")
    out = {"workload": "R-MAT scale 22 edge factor 16, window %d edges; %d slides of %d deletes + %d inserts"
                       % (st.window, slides, b, b)}
    arrivals = st.order[st.window:]
    expiry = [st.slide(t, b) for t in range(slides)]
    cases = {
        "explicit_random_deletions": (synth.explicit_deletion_slides(st.initial(), arrivals, b, slides,
                                                                     args.seed + 41), False),
        "sorted_arrivals": ([synth.sorted_stream(st).slide(t, b) for t in range(slides)], False),
        "window_expiry_merged_deletes": (expiry, False),
        "window_expiry_lazy_deletes": (expiry, True),
    }
    for name, (sl, lazy) in cases.items():
        res = {}
        handles = {}
        for mode in ("plain", "fused"):
            g = GPMA(st.V, st.initial(), mirror=True, learned=(mode == "fused"), lazy_delete=lazy)
            d0, i0 = sl[0]
            if mode == "fused":
                g.apply_batches([1, 0], [d0, i0])
            else:
                g.delete(d0)
                g.insert(i0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = 0
            for d, i in sl[1:]:
                if mode == "fused":
                    n += g.apply_batches([1, 0], [d, i]).applied
                else:
                    n += g.delete(d, stats=True).applied + g.insert(i, stats=True).applied
            torch.cuda.synchronize()
            res[mode + "_updates_per_s"] = n / (time.perf_counter() - t0)
            handles[mode] = g
        res["fused_speedup"] = res["fused_updates_per_s"] / res["plain_updates_per_s"]
        res["identical_output"] = bool(torch.equal(handles["plain"].slots(), handles["fused"].slots()))
        if lazy:
            s = handles["fused"].slots()
            res["marked_entries"] = int(((s < 0) & (s != -1)).sum().item())
        for g in handles.values():
            g.close()
        out[name] = res
        log("%s: %s" % (name, res))
    return out


def service_section(args):
    """Streaming service on R-MAT scale 22 (window = first half of the
    distinct edges): for each rate, Poisson edge arrivals for `service_s`
    seconds with continuous batching, BFS and 10-iteration PageRank queries at
    a Poisson rate, the graph and the query slots under one HBM budget; then
    a saturated run (every edge already arrived, the update stream applies
    steps back to back) for the sustained update throughput beside queries."""
    import torch

    import synth
    from paper_1709_05061_amd.service import GraphService
    st = synth.rmat_stream(22, 16, seed=args.seed + 30, device="cuda")
    V = st.V
    out = {"workload": "R-MAT scale 22 edge factor 16, window %d edges; Poisson arrivals for %gs per rate; "
                       "BFS + PageRank(10) queries at %g/s; HBM budget %d GiB for graph and query slots"
                       % (st.window, args.service_s, args.query_rate, args.service_budget_gib),
           "rates": {}}
    pos = st.window
    cases = [(1e5, False), (1e6, False), (1e7, False), (None, True)]
    for k, (rate, saturated) in enumerate(cases):
        if saturated:
            n = min(1 << 22, st.order.numel() - pos)
            times = torch.zeros(n, dtype=torch.float64)
        else:
            # (at most 2e7 arrivals, so the saturated run still has 4M left)
            n = min(int(rate * args.service_s), 20_000_000, st.order.numel() - pos)
            times = synth.poisson_times(n, rate, seed=args.seed + 31 + k)
        arrivals = st.order[pos:pos + n]
        nq = max(4, int(args.query_rate * args.service_s))
        qt = synth.poisson_times(nq, args.query_rate, seed=args.seed + 41 + k).tolist()
        kinds = ["bfs" if i % 2 == 0 else "pagerank" for i in range(nq)]
        srcs = synth.uniform_below(torch.arange(nq), args.seed + 51 + k, V).tolist()
        qargs = [srcs[i] if kinds[i] == "bfs" else 10 for i in range(nq)]
        window = st.order[pos - st.window:pos]
        svc = GraphService(V, window, mirror=True, hbm_budget_bytes=args.service_budget_gib << 30,
                           max_batch=1 << 18, max_slots=4)
        rep = svc.run(times, arrivals, qt, kinds, qargs, time_limit_s=120)
        name = "saturated" if saturated else "%g" % rate
        out["rates"][name] = rep.summary()
        log("service %s: %s" % (name, rep.summary()))
        svc.close()
        del svc
        torch.cuda.empty_cache()
        pos += n
    return out


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
    ap.add_argument("--plain", action="store_true", help="time the plain per-batch path as value")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-path comparison run")
    ap.add_argument("--uneven-slides", type=int, default=128)
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-service", action="store_true")
    ap.add_argument("--no-workloads", action="store_true", help="skip the explicit-deletion / sorted-stream section")
    ap.add_argument("--rebuild-slides", type=int, default=4, help="slides timed on the rebuild-per-batch CSR")
    ap.add_argument("--lock-slides", type=int, default=4,
                    help="slides timed for the lock-based GPMA comparator (0: skip)")
    ap.add_argument("--service-s", type=float, default=5.0)
    ap.add_argument("--query-rate", type=float, default=200.0)
    ap.add_argument("--service-budget-gib", type=int, default=16)
    ap.add_argument("--no-learned", action="store_true", help="binary-search locate in the main path")
    ap.add_argument("--fused-direct", type=int, default=0,
                    help="1: fused batches enqueue their kernels directly, 0: replay captured graphs")
    ap.add_argument("--sort-tile", type=int, default=1024, help="keys per batch-sort workgroup tile")
    ap.add_argument("--fused-levels", type=int, default=0,
                    help="tree levels above the leaves each fused batch runs on the device")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slides", type=int, default=2, help="slides through the layout oracle")
    ap.add_argument("--cpu-set-slides", type=int, default=4, help="slides through the sorted-vector set")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--sweep", default="1,16,256,1024,4096,16384,65536,262144,1048576",
                    help="batch sizes of the latency sweep (fused + learned, fused + binary search, plain)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--spmv", default="auto", help="SpMV form of the headline handle (a key of SPMV_FORMS)")
    ap.add_argument("--no-spmv-forms", action="store_true", help="skip timing the other binned SpMV form")
    ap.add_argument("--no-resize", action="store_true", help="skip the scale-24 root doubling")
    ap.add_argument("--no-rmat20", action="store_true", help="skip the scale-20 batch-size section")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (4 launches), the known-size reference "
                         "for hardware byte counters, and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the PMA would shard by vertex range; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd import gpma as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # an elementwise kernel that reads 2^27 int64 and writes 2^27 int64
        src = torch.arange(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"read_bytes": 8 << 27, "write_bytes": 8 << 27,
                                               "launches": 4}}))
        return
    b = args.batch
    sweep = [] if args.no_sweep else [int(x) for x in args.sweep.split(",")]
    need = (args.warmup + args.steps) * b + sum(sweep_slides(z) * z for z in sweep)
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
    mirror = not args.no_mirror
    fused_mode = not args.plain
    t0 = time.time()
    learned = not args.no_learned
    g = GPMA(V, st.initial(), leaf_size=args.leaf_size, mirror=mirror, learned=learned,
             fused_direct=bool(args.fused_direct), sort_tile=args.sort_tile, fused_levels=args.fused_levels,
             spmv=args.spmv)
    torch.cuda.synchronize()
    log("created PMA: %d edges, capacity %d slots, leaf %d in %.1fs"
        % (g.num_edges, g.capacity, g.leaf_size, time.time() - t0))
    stream = torch.cuda.current_stream()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def byte_rates(h):
        # per handle, looked up once (outside the timed calls after the first):
        # bytes per rewritten slot, and the handles (array, mirror)
        r = getattr(h, "_bench_rates", None)
        if r is None:
            r = (16.0 + 10.0 / h.leaf_size, 2 if h.mirror() is not None else 1)
            h._bench_rates = r
        return r

    def update(h, t, fused, bsz=None, t0=0):
        """One slide; returns (applied, resizes, algorithmic bytes): per
        handle 8 B per batch key plus, per merged segment, 16 B per slot and
        10 B per leaf (read and written slots, leaf counts), over the array
        and its mirror."""
        d, i = st.slide(t, b) if bsz is None else (st.order[t0:t0 + bsz],
                                                  st.order[st.window + t0: st.window + t0 + bsz])
        per_slot, nh = byte_rates(h)
        if fused:
            s = h.apply_batches([1, 0], [d, i])
            by = nh * 8.0 * (d.numel() + i.numel()) + per_slot * (s.slots_rewritten + s.mirror_slots_rewritten)
            return s.applied, int(s.resized), by
        sd = h.delete(d, stats=True)
        si = h.insert(i, stats=True)
        rw = sd.slots_rewritten + sd.mirror_slots_rewritten + si.slots_rewritten + si.mirror_slots_rewritten
        by = nh * 8.0 * (d.numel() + i.numel()) + per_slot * rw
        return sd.applied + si.applied, int(sd.resized) + int(si.resized), by

    # the other update path on a second handle, same slides: throughput and
    # identical output
    other = None
    other_ups = None
    if not args.no_compare:
        # the baseline path: plain per-batch calls, binary-search locate
        other = GPMA(V, st.initial(), leaf_size=args.leaf_size, mirror=mirror)
        for t in range(args.warmup):
            update(other, t, not fused_mode)
        ms = []
        n_o = 0
        for t in range(args.warmup, args.warmup + args.steps):
            e0 = ev()
            a, _, _ = update(other, t, not fused_mode)
            e1 = ev()
            n_o += a
            ms.append((e0, e1))
        torch.cuda.synchronize()
        other_ups = n_o / (sum(a.elapsed_time(c) for a, c in ms) / 1e3)
        log("%s path: %.3g updates/s" % ("plain" if fused_mode else "fused", other_ups))

    # the headline configuration with lazy deletion (the paper's experimental
    # setup for GPMA and GPMA+: expired edges are marked, not merged out)
    lazy_ups = None
    if not args.no_compare:
        h = GPMA(V, st.initial(), leaf_size=args.leaf_size, mirror=mirror, learned=learned,
                 fused_direct=bool(args.fused_direct), sort_tile=args.sort_tile, fused_levels=args.fused_levels,
                 lazy_delete=True)
        for t in range(args.warmup):
            update(h, t, fused_mode)
        ms = []
        n_z = 0
        for t in range(args.warmup, args.warmup + args.steps):
            e0 = ev()
            a, _, _ = update(h, t, fused_mode)
            e1 = ev()
            n_z += a
            ms.append((e0, e1))
        torch.cuda.synchronize()
        lazy_ups = n_z / (sum(a.elapsed_time(c) for a, c in ms) / 1e3)
        log("same path with lazy deletes: %.3g updates/s" % lazy_ups)
        h.close()
        del h
        torch.cuda.empty_cache()

    # comparator: a CSR rebuilt on every batch (the paper's GPU-CSR baseline
    # role), on the first slides
    rebuild = None
    if not args.no_compare and args.rebuild_slides > 0:
        from paper_1709_05061_amd import CSRRebuild
        c = CSRRebuild(V, st.initial())
        d, i = st.slide(0, b)
        c.delete(d)
        c.insert(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, 1 + args.rebuild_slides):
            d, i = st.slide(t, b)
            c.delete(d)
            c.insert(i)
        torch.cuda.synchronize()
        rebuild = {"updates_per_s": 2 * b * args.rebuild_slides / (time.perf_counter() - t0),
                   "slides": args.rebuild_slides, "edges": c.num_edges}
        c.close()
        del c
        torch.cuda.empty_cache()
        log("CSR rebuilt per batch: %.3g updates/s" % rebuild["updates_per_s"])

    # comparator: the lock-based GPMA (one insertion per worker, per-height
    # try-locks, retries in rounds) against GPMA+ (plain per-batch calls), both
    # with lazy deletion as in the paper's experiments, on the first slides
    lock = None
    if not args.no_compare and args.lock_slides > 0:
        lock = {"slides": args.lock_slides}
        for name in ("gpma_plus", "gpma_lock"):
            h = GPMA(V, st.initial(), leaf_size=args.leaf_size, lazy_delete=True)
            rounds = []
            d, i = st.slide(0, b)
            h.delete(d)
            if name == "gpma_lock":
                h.lock_insert(i)
            else:
                h.insert(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n_l = 0
            for t in range(1, 1 + args.lock_slides):
                d, i = st.slide(t, b)
                n_l += h.delete(d, stats=True).applied
                if name == "gpma_lock":
                    si, r = h.lock_insert(i)
                    rounds.append(r)
                else:
                    si = h.insert(i, stats=True)
                n_l += si.applied
            torch.cuda.synchronize()
            lock[name + "_updates_per_s"] = n_l / (time.perf_counter() - t0)
            if rounds:
                lock["lock_rounds_per_insert_batch"] = rounds
            log("%s with lazy deletes: %.3g updates/s%s" % (name, lock[name + "_updates_per_s"],
                                                             (", rounds %s" % rounds) if rounds else ""))
            h.close()
            del h
            torch.cuda.empty_cache()
        lock["gpma_plus_speedup"] = lock["gpma_plus_updates_per_s"] / lock["gpma_lock_updates_per_s"]

    # BFS sources: vertices with out-edges, drawn with the seeded generator
    deg = g.degrees()
    cand = torch.nonzero(deg > 0).flatten()
    pick = synth.uniform_below(torch.arange(args.warmup + args.steps, device="cuda"), args.seed + 7,
                               cand.numel())
    sources = cand[pick].tolist()
    x = torch.full((V,), 1.0 / V, dtype=torch.float32, device="cuda")

    def step(t):
        e0 = ev()
        a, r, by = update(g, t, fused_mode)
        e1 = ev()
        marks = [e0, e1, by]
        if not args.no_analytics:
            g.pagerank(init=x, iters=args.pr_iters, out=x)
            marks.append(ev())
            dist = g.bfs(sources[t])
            marks.append(ev())
            g.cc()
            marks.append(ev())
            # BFS algorithmic bytes: 8 B per slot of every reached row, 12 B per vertex
            ro = g.row_offsets().to(torch.int64)
            marks.append(8.0 * float(((ro[1:] - ro[:-1])[dist >= 0]).sum().item()) + 12.0 * V)
        return a, r, marks

    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    loc0 = g.locator_info() if learned else None
    g.profile_reset()
    g.profile(True)
    recs = []
    applied = 0
    resized = 0
    torch.cuda.synchronize()
    tw0 = time.perf_counter()
    for t in range(args.warmup, args.warmup + args.steps):
        a, r, marks = step(t)
        applied += a
        resized += r
        recs.append(marks)
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw0
    g.profile(False)

    upd_ms = [m[0].elapsed_time(m[1]) for m in recs]
    upd_bytes = sum(m[2] for m in recs)
    phases = {"update": sum(upd_ms) / len(recs)}
    if not args.no_analytics:
        phases["pagerank"] = sum(m[1].elapsed_time(m[3]) for m in recs) / len(recs)
        phases["bfs"] = sum(m[3].elapsed_time(m[4]) for m in recs) / len(recs)
        phases["cc"] = sum(m[4].elapsed_time(m[5]) for m in recs) / len(recs)
    updates_per_s = applied / (sum(upd_ms) / 1e3)
    upd_gbps = upd_bytes / (sum(upd_ms) / 1e3) / 1e9
    roofline_update = {"bound": "hbm", "achieved": upd_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": upd_gbps / HBM_PEAK_GBPS, "traffic": None,
                       "bytes_per_slide": upd_bytes / len(recs),
                       "note": "whole update phase (every kernel of a slide, array and mirror) against "
                               "8 B per batch key + (16 + 10/leaf) B per slot of every merged segment"}
    roofline_bfs = None
    if not args.no_analytics:
        bfs_ms = [m[3].elapsed_time(m[4]) for m in recs]
        bfs_gbps = sum(m[6] for m in recs) / (sum(bfs_ms) / 1e3) / 1e9
        roofline_bfs = {"bound": "hbm", "achieved": bfs_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": bfs_gbps / HBM_PEAK_GBPS, "traffic": None,
                        "bytes_per_bfs": sum(m[6] for m in recs) / len(recs),
                        "note": "whole BFS call against 8 B per slot of every reached row + 12 B per vertex"}
    loc_timed = None
    if learned:
        loc1 = g.locator_info()
        loc_timed = {"fits": loc1["fits"] - loc0["fits"], "lookups": loc1["lookups"] - loc0["lookups"],
                     "misses": loc1["misses"] - loc0["misses"], "eps": loc1["eps"]}

    # latency against batch size (the paper's update experiment, Section 6.2):
    # the same slides on the headline handle (fused + learned locator), on a
    # fused handle with binary-search locate and on the plain handle
    sweep_out = None
    if sweep and other is not None and fused_mode:
        log("batch-size sweep %s" % sweep)
        fb = GPMA(V, st.initial(), leaf_size=args.leaf_size, mirror=mirror, learned=False,
                  fused_direct=bool(args.fused_direct), sort_tile=args.sort_tile, fused_levels=args.fused_levels)
        for t in range(args.warmup + args.steps):   # catch up with the headline handle
            update(fb, t, True)
        paths = {"fused_learned": (g, True), "fused_binary": (fb, True), "plain": (other, False)}
        sweep_out = {"sizes": sweep, "slides": [], **{k: {"ms_per_slide": [], "updates_per_s": []} for k in paths}}
        t0 = (args.warmup + args.steps) * b
        for z in sweep:
            k = sweep_slides(z)
            for name, (h, fz) in paths.items():
                update(h, 0, fz, bsz=z, t0=t0)            # warm-up slide: graphs for this size class
                marks, n = [], 0
                for j in range(1, k):
                    e0 = ev()
                    a, _, _ = update(h, 0, fz, bsz=z, t0=t0 + j * z)
                    e1 = ev()
                    n += a
                    marks.append((e0, e1))
                torch.cuda.synchronize()
                ms = sum(x.elapsed_time(y) for x, y in marks) / len(marks)
                sweep_out[name]["ms_per_slide"].append(ms)
                sweep_out[name]["updates_per_s"].append(n / len(marks) / (ms / 1e3))
            sweep_out["slides"].append(k - 1)
            log("b=%d: %s" % (z, {name: "%.3f ms" % sweep_out[name]["ms_per_slide"][-1] for name in paths}))
            t0 += k * z
        sweep_out["learned_over_binary"] = [a / c for a, c in zip(sweep_out["fused_learned"]["updates_per_s"],
                                                                   sweep_out["fused_binary"]["updates_per_s"])]
        sweep_out["fused_over_plain"] = [a / c for a, c in zip(sweep_out["fused_learned"]["updates_per_s"],
                                                                sweep_out["plain"]["updates_per_s"])]
        sweep_out["identical_output"] = bool(torch.equal(g.slots(), fb.slots()) and torch.equal(g.slots(),
                                                                                                other.slots()))
        if learned:
            sweep_out["locator"] = g.locator_info()
        fb.close()
        del fb
        torch.cuda.empty_cache()

    identical = None
    if other is not None:
        identical = bool(torch.equal(g.slots(), other.slots()))
        if mirror:
            identical = identical and bool(torch.equal(g.mirror().slots(), other.mirror().slots()))
        other.close()
        del other

    kernels = {}
    for kid, name in enumerate(G.KERNEL_NAMES):
        ms, n, by = g.profile_read(kid)
        if n:
            kernels[name] = {"launches": n, "mean_us": 1e3 * ms / n, "total_ms": ms,
                             "GBps": (by / (ms / 1e3) / 1e9) if by and ms else None}
    roofline = None
    if kernels:
        dom_name, dom_k = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
        achieved = dom_k["GBps"]
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": (achieved / HBM_PEAK_GBPS) if achieved else None,
                    "traffic": measured_traffic(dom_name), "kernel": dom_name}
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
                   "mirror": mirror, "update_path": "fused" if fused_mode else "plain",
                   "fused_direct": bool(args.fused_direct), "sort_tile": args.sort_tile,
                   "fused_levels": args.fused_levels,
                   "learned_locator": learned},
        "phases_ms": phases,
        "update_ms_p50": pctl(upd_ms, 50),
        "update_ms_p99": pctl(upd_ms, 99),
        "applied_per_step": applied / args.steps,
        "resizes": resized,
        ("plain_updates_per_s" if fused_mode else "fused_updates_per_s"): other_ups,
        "csr_rebuild": rebuild,
        "lock_gpma": lock,
        "lazy_delete_updates_per_s": lazy_ups,
        "fused_speedup": (updates_per_s / other_ups if fused_mode else other_ups / updates_per_s)
        if other_ups else None,
        "identical_output": identical,
        "spmv_GBps": spmv["GBps"] if spmv else None,
        "spmv_frac": (spmv["GBps"] / HBM_PEAK_GBPS) if spmv and spmv["GBps"] else None,
        "kernels": kernels,
        "roofline": roofline,
        "roofline_update": roofline_update,
        "roofline_bfs": roofline_bfs,
        "batch_sweep": sweep_out,
    }
    if learned:
        out["locator"] = g.locator_info()
        out["locator_timed_steps"] = loc_timed
    if mirror and fused_mode:
        # 1: the array's pipeline on the caller's stream, the mirror's beside
        # it; 0: both on handle streams (forked and joined)
        out["fused_pairing"] = g.fused_pairing()
    if not args.no_spmv_forms:
        out["spmv_forms"] = spmv_forms_section(args, g, st, V, kernels)
    g.close()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the headline inputs")
        out["cpu_baseline"] = cpu_baseline(st, b, args.cpu_slides, args.cpu_set_slides)
    else:
        out["cpu_baseline"] = None
    del st
    torch.cuda.empty_cache()
    if not args.no_service:
        log("streaming service (R-MAT scale 22)")
        out["service"] = service_section(args)
        r7 = out["service"]["rates"].get("1e+07") or {}
        out["stream_latency_ms_p99"] = r7.get("edge_latency_ms_p99")
        torch.cuda.empty_cache()
    if not args.no_resize:
        log("root doubling at scale 24")
        out["resize"] = resize_section(args)
        log("resize: %s" % out["resize"])
        torch.cuda.empty_cache()
    if not args.no_rmat20:
        log("R-MAT scale 20 batch sizes with analytics")
        out["rmat20"] = rmat20_section(args)
        torch.cuda.empty_cache()
    if not args.no_uneven:
        log("uneven-batch workload (power-law graph)")
        out["uneven"] = uneven_section(args)
        torch.cuda.empty_cache()
    if not args.no_workloads:
        log("explicit deletions and sorted arrivals (R-MAT scale 22)")
        out["workloads"] = workloads_section(args)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
