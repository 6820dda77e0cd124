#!/usr/bin/env python3
"""Benchmark: cooperative vs plain persistent BFS on R-MAT scale 22, with the
co-task preemption measurement.

Workload (one GPU): R-MAT scale 22, edge factor 16 (a=0.57, b=0.19,
c=0.19, d=0.05), seeded, permuted, symmetrised, loops/duplicates removed,
uint32 CSR resident in HBM. A *step* is one BFS traversal from the next
seeded source (degree >= 1) inside one persistent cooperative launch
(the scheduler target word is polled at every resizing barrier, kept at N).

Printed JSON line (one):
  value          GTEPS of the cooperative launch: sum over sources of the
                 undirected edges in the source's component / time
  plain          same sources in a plain persistent launch (fixed M)
  coop_overhead  cooperative time / plain time
  cotask         a co-task every 10 ms needing half the CUs for 1 ms while
                 a cooperative launch runs: p50/p99 latency, gather time,
                 slowdown of the traversal
  roofline       algorithmic bytes of the traversal / kernel time vs 8 TB/s
  cpu_baseline   the oracle's FIFO BFS on the host, bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--cotask-seconds", type=float, default=2.0)
    ap.add_argument("--cpu-sample", type=int, default=4, help="sources for the oracle timing")
    ap.add_argument("--skip-cotask", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1707_01989_amd import coop, graphgen as gg

    t0 = time.time()
    g = gg.rmat(args.scale, 16, seed=3)
    log(f"rmat{args.scale}: n={g.n} arcs={g.arcs} generated in {time.time() - t0:.1f}s")
    deg = g.degrees()
    nsrc = args.warmup + args.steps
    roots = gg.sources(g, 3, nsrc)

    # per-source traversal sizes for GTEPS and algorithmic bytes (component
    # of each source: undirected edges, vertices reached)
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    A = csr_matrix((np.ones(g.arcs, dtype=np.int8), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                   shape=(g.n, g.n))
    _, comp = connected_components(A, directed=False)
    comp_edges = np.bincount(comp, weights=deg, minlength=comp.max() + 1) / 2
    comp_verts = np.bincount(comp, minlength=comp.max() + 1)
    edges_of = lambda r: float(comp_edges[comp[r]])
    verts_of = lambda r: int(comp_verts[comp[r]])

    rt = coop.Runtime(0)
    dg = rt.graph(g)
    timed = roots[args.warmup:]
    d_warm = rt._roots(roots[:args.warmup])
    d_timed = rt._roots(timed)
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(mode_opts, d_roots, k):
        h = coop.coop_bfs(rt.rt, dg.handle, d_roots, k, level, 0, mode_opts, stream)
        rc, st = coop.coop_wait(h)
        if rc != 0:
            raise RuntimeError(coop.coop_strerror(rc))
        return st

    coop_opts = coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_HOST_SCHEDULE)
    plain_opts = coop.make_opts(coop.COOP_MODE_PLAIN)
    # warmup
    run(coop_opts, d_warm, args.warmup)
    run(plain_opts, d_warm, args.warmup)
    torch.cuda.synchronize()

    edges = sum(edges_of(int(r)) for r in timed)
    verts = sum(verts_of(int(r)) for r in timed)
    arcs_scanned = 2 * edges
    # algorithmic bytes (top-down frontier BFS): per scanned arc 4 B column
    # index + 4 B visited probe; per reached vertex 8 B row range, 4 B
    # frontier read, 4 B frontier write, 4 B level write; per source the
    # level and visited-set initialisation (4 B + 1/8 B per vertex)
    alg_bytes = 8 * arcs_scanned + 20 * verts + len(timed) * (4.125 * g.n)

    t = time.perf_counter()
    st_c = run(coop_opts, d_timed, len(timed))
    torch.cuda.synchronize()
    wall_c = time.perf_counter() - t
    t = time.perf_counter()
    st_p = run(plain_opts, d_timed, len(timed))
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t
    ms_c, ms_p = st_c["kernel_ms"], st_p["kernel_ms"]
    log(f"coop {ms_c:.3f} ms (wall {wall_c*1e3:.1f}), plain {ms_p:.3f} ms, levels {st_c['levels']}")

    gteps_c = edges / (ms_c * 1e-3) / 1e9
    gteps_p = edges / (ms_p * 1e-3) / 1e9
    achieved = alg_bytes / (ms_c * 1e-3) / 1e9

    result = {
        "metric": "GTEPS BFS/SSSP coop vs plain persistent kernel; p99 co-task latency",
        "value": round(gteps_c, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_c / len(timed), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"BFS on R-MAT scale {args.scale} (edge factor 16, a=.57 b=.19 c=.19), "
                               f"one source per step, one persistent cooperative launch",
                   "n": g.n, "arcs": g.arcs, "sources": len(timed), "parallelism": "1 GPU",
                   "groups": st_c["grid"], "group_size": 1024},
        "plain": {"value": round(gteps_p, 3), "ms": round(ms_p, 3)},
        "coop_overhead": round(ms_c / ms_p, 4),
        "barriers": st_c["barriers"],
    }

    if not args.skip_cotask:
        # co-task every 10 ms needing half the CUs for 1 ms during a long launch
        per_root_ms = ms_c / len(timed)
        k = max(1, int(args.cotask_seconds * 1e3 / max(per_root_ms, 1e-3)))
        k = min(k, 200000)
        reps = np.resize(timed, k)
        d_many = rt._roots(reps)
        alone = run(coop_opts, d_many, k)
        cus = rt.info["compute_units"]
        h = coop.coop_bfs(rt.rt, dg.handle, d_many, k, level, 0, coop_opts, stream)
        coop.coop_injector_start(rt.rt, h, groups=cus // 2, busy_ns=1_000_000, period_ns=10_000_000)
        rc, st_m = coop.coop_wait(h)
        irc, cst = coop.coop_injector_stop(rt.rt)
        if rc != 0 or irc != 0:
            raise RuntimeError(f"co-task run failed: {coop.coop_strerror(rc)} / {coop.coop_strerror(irc)}")
        result["cotask"] = {
            "period_ms": 10, "busy_ms": 1, "groups": cus // 2, "count": cst["count"],
            "latency_p50_ms": round(cst["latency_p50_ms"], 4), "latency_p99_ms": round(cst["latency_p99_ms"], 4),
            "gather_p50_ms": round(cst["gather_p50_ms"], 4), "gather_p99_ms": round(cst["gather_p99_ms"], 4),
            "slowdown": round(st_m["kernel_ms"] / alone["kernel_ms"], 4),
            "kills": st_m["kills"], "forks": st_m["forks"],
            "model_kernel_preemption": round(10 / 9, 4), "model_half_cu": round(10 / 9.5, 4),
        }
        log(f"cotask: {result['cotask']}")

    result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                          "kernel": "bfs_kernel<true>", "alg_bytes_per_launch": int(alg_bytes)}

    # CPU baseline: the oracle (single-threaded FIFO BFS) on a bounded sample
    import oracle
    sample = [int(r) for r in timed[:args.cpu_sample]]
    t = time.perf_counter()
    for r in sample:
        oracle.bfs(g, r)
    cpu_s = time.perf_counter() - t
    cpu_edges = sum(edges_of(r) for r in sample)
    result["cpu_baseline"] = {"value": round(cpu_edges / cpu_s / 1e9, 5), "unit": "GTEPS", "cores": 1,
                              "kind": "oracle", "sample": f"{len(sample)} sources of the same graph, "
                                                          f"{cpu_s:.2f} s"}
    rt.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
