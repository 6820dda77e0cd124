#!/usr/bin/env python3
"""Benchmark: cooperative vs plain persistent BFS on R-MAT scale 22, with the
co-task preemption measurement and an SSSP grid side line.

Workload (one GPU): R-MAT scale 22, edge factor 16 (a=0.57, b=0.19,
c=0.19, d=0.05), seeded, permuted, symmetrised, loops/duplicates removed,
uint32 CSR resident in HBM. A *step* is one BFS traversal from the next
seeded source (degree >= 1). Steps run inside persistent cooperative
launches of ``--roots-per-launch`` sources each (the scheduler target word
is polled at every resizing barrier and kept at N), so every launch of the
kernel does the same kind of work and the per-launch event time can be
compared with a profiler's per-dispatch average.

Printed JSON line (one):
  value          GTEPS of the cooperative launches: sum over sources of the
                 undirected edges in the source's component / wall time of
                 the timed region (synchronised on both sides)
  plain          same sources in plain persistent launches (fixed M)
  coop_overhead  cooperative time / plain time (kernel events)
  sssp           frontier Bellman-Ford on the 1024x1024 grid, coop vs plain,
                 and one run under a seeded random kill/fork schedule
  cotask         a co-task every 10 ms needing half the CUs for 1 ms while
                 a cooperative launch runs: p50/p99 latency, gather time,
                 slowdown of the traversal
  shared         a long cooperative BFS and the SSSP grid launched together,
                 the host sharer splitting the resident workgroups between
                 them: each one's time alone and shared, wall time shared
  octree         work-stealing octree build (4M clustered points): coop vs
                 plain, and co-task latency during one build
  gather_sweep   gather time against the workgroups a co-task claims (1, a
                 quarter, half, all but one), query barrier vs the regular
                 barrier that lets one workgroup go per barrier
  roofline       algorithmic bytes per launch / mean launch time (HIP events
                 on the launch stream) vs 8 TB/s; traffic from the committed
                 PMC summary when it was taken on the current kernel sources
  cpu_baseline   the oracle's FIFO BFS on the host, bounded sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bfs_kernel_rmat22_traffic.txt")
# the kernel and the runtime that sizes and parameterises its launches
KERNEL_SOURCES = ("paper_1707_01989_amd/csrc/coop_kernels.hip", "paper_1707_01989_amd/csrc/traverse.h",
                  "paper_1707_01989_amd/csrc/coop_internal.h", "include/coop_device.hpp",
                  "paper_1707_01989_amd/csrc/coop_runtime.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per launch from the committed PMC summary, or None when the
    summary is missing or was taken on other kernel sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"^source_hash:\s*(\w+)", text, re.M)
    b = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--roots-per-launch", type=int, default=8)
    ap.add_argument("--cotask-seconds", type=float, default=4.0)
    ap.add_argument("--gather-seconds", type=float, default=0.5, help="per point of the gather-time sweep")
    ap.add_argument("--cpu-sample", type=int, default=32, help="sources for the oracle timing")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one int32 'x + 1' elementwise kernel over this many MiB (counter calibration)")
    ap.add_argument("--skip-cotask", action="store_true")
    ap.add_argument("--skip-sssp", action="store_true")
    ap.add_argument("--skip-share", action="store_true")
    ap.add_argument("--skip-octree", action="store_true")
    ap.add_argument("--barrier-bench-plain", action="store_true",
                    help="also time 2000 barriers of an empty plain persistent launch (off by default: "
                         "one such run waited out its watchdog under the profiler)")
    ap.add_argument("--skip-barrier", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    L = max(1, args.roots_per_launch)
    if args.steps % L or args.warmup % L:
        sys.exit(f"--steps and --warmup must be multiples of --roots-per-launch ({L})")

    import numpy as np
    import torch

    from paper_1707_01989_amd import coop, graphgen as gg

    t0 = time.time()
    g = gg.rmat(args.scale, 16, seed=3)
    log(f"rmat{args.scale}: n={g.n} arcs={g.arcs} generated in {time.time() - t0:.1f}s")
    deg = g.degrees()
    roots = gg.sources(g, 3, args.warmup + args.steps)

    # per-source traversal sizes (component of each source)
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
    timed = [int(r) for r in roots[args.warmup:]]
    batches_w = [rt._roots(roots[i:i + L]) for i in range(0, args.warmup, L)]
    batches_t = [rt._roots(timed[i:i + L]) for i in range(0, args.steps, L)]
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(opts, d_roots):
        h = coop.coop_bfs(rt.rt, dg.handle, d_roots, d_roots.numel(), level, 0, opts, stream)
        rc, st = coop.coop_wait(h)
        if rc != 0:
            raise RuntimeError(coop.coop_strerror(rc))
        return st

    coop_opts = coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_HOST_SCHEDULE)
    plain_opts = coop.make_opts(coop.COOP_MODE_PLAIN)
    for b in batches_w:
        run(coop_opts, b)
        run(plain_opts, b)
    torch.cuda.synchronize()

    def timed_region(opts):
        # every launch is queued on the stream before the first is waited
        # for, as a caller streaming sources would do: the launches run back
        # to back and the host collects each one's statistics meanwhile
        torch.cuda.synchronize()
        t = time.perf_counter()
        hs = [coop.coop_bfs(rt.rt, dg.handle, b, b.numel(), level, 0, opts, stream) for b in batches_t]
        sts = []
        for h in hs:
            rc, st = coop.coop_wait(h)
            if rc != 0:
                raise RuntimeError(coop.coop_strerror(rc))
            sts.append(st)
        torch.cuda.synchronize()
        return time.perf_counter() - t, sts

    wall_c, sts_c = timed_region(coop_opts)
    wall_p, sts_p = timed_region(plain_opts)
    ms_c = sum(s["kernel_ms"] for s in sts_c)
    ms_p = sum(s["kernel_ms"] for s in sts_p)
    launch_ms = ms_c / len(sts_c)
    log(f"coop {ms_c:.3f} ms kernel / {wall_c*1e3:.1f} ms wall, plain {ms_p:.3f} / {wall_p*1e3:.1f}; "
        f"launch mean {launch_ms:.3f} ms, levels {sum(s['levels'] for s in sts_c)}")

    edges = sum(edges_of(r) for r in timed)
    verts = sum(verts_of(r) for r in timed)
    gteps_c = edges / wall_c / 1e9
    gteps_p = edges / wall_p / 1e9

    # algorithmic bytes of a level-synchronous BFS, at the data's natural
    # width: 8 B per scanned arc (column index + state probe) and 20 B per
    # reached vertex (row range, frontier read and write, level write);
    # arcs scanned = the degree sum of the reached vertices
    alg_bytes_launch = (8 * 2 * edges + 20 * verts) / len(sts_c)
    achieved = alg_bytes_launch / (launch_ms * 1e-3) / 1e9
    # what this kernel itself read, by its own counters (direction-optimising
    # BFS skips arcs): 4 B per arc examined, 8 B per row range, 4 B per
    # bitmap word, summed over the timed launches
    counted = sum(4 * s["arcs"] + 8 * s["rows"] + 4 * s["bitmap_words"] for s in sts_c) / len(sts_c)

    result = {
        "metric": "GTEPS BFS/SSSP coop vs plain persistent kernel; p99 co-task latency",
        "value": round(gteps_c, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_c * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"BFS on R-MAT scale {args.scale} (edge factor 16, a=.57 b=.19 c=.19, seed 3), "
                               f"one seeded source per step, {L} sources per persistent cooperative launch, "
                               f"co-task every 10 ms needing half the CUs for 1 ms",
                   "n": g.n, "arcs": g.arcs, "sources": len(timed), "roots_per_launch": L,
                   "groups": sts_c[0]["grid"], "group_size": 1024},
        "plain": {"value": round(gteps_p, 3), "kernel_ms": round(ms_p, 3), "wall_ms": round(wall_p * 1e3, 3)},
        "coop_overhead": round(ms_c / ms_p, 4),
        "kernel_ms": round(ms_c, 3),
        "barriers": sum(s["barriers"] for s in sts_c),
    }

    if not args.skip_sssp:
        # frontier Bellman-Ford on the 1024x1024 grid, w U[1,1000], source 0
        gs = gg.add_weights(gg.grid(1024, 1024), 2, 1, 1000)
        dgs = rt.graph(gs)
        dist = torch.empty(gs.n, dtype=torch.int32, device="cuda")
        d0 = rt._roots([0])

        def run_s(opts):
            h = coop.coop_sssp(rt.rt, dgs.handle, d0, 1, dist, 0, opts, stream)
            rc, st = coop.coop_wait(h)
            if rc != 0:
                raise RuntimeError(coop.coop_strerror(rc))
            return st
        run_s(coop_opts)
        run_s(plain_opts)
        reps = 5
        sc = [run_s(coop_opts)["kernel_ms"] for _ in range(reps)]
        sp = [run_s(plain_opts)["kernel_ms"] for _ in range(reps)]
        rnd = coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_RANDOM_SCHEDULE | coop.COOP_F_PARK_KILLED,
                             sched_seed=1, sched_p=0.25)
        st_r = run_s(rnd)
        ref = dist.clone()
        st_1 = run_s(coop_opts)
        same = bool(torch.equal(ref, dist))
        e_s = gs.edges
        result["sssp"] = {
            "workload": "frontier Bellman-Ford, 1024x1024 grid, w U[1,1000] (seed 2), source 0",
            "gteps_coop": round(e_s / (np.median(sc) * 1e-3) / 1e9, 4),
            "gteps_plain": round(e_s / (np.median(sp) * 1e-3) / 1e9, 4),
            "ms_coop": round(float(np.median(sc)), 3), "ms_plain": round(float(np.median(sp)), 3),
            "coop_overhead": round(float(np.median(sc) / np.median(sp)), 4),
            "rounds": st_1["barriers"],
            "ns_per_barrier_coop": round(float(np.median(sc)) * 1e6 / st_1["barriers"], 1),
            "random_schedule": {"seed": 1, "p": 0.25, "ms": round(st_r["kernel_ms"], 3), "kills": st_r["kills"],
                                "forks": st_r["forks"], "min_groups": st_r["min_groups"],
                                "same_as_never_resize": same},
        }
        log(f"sssp: {result['sssp']}")

    if not args.skip_cotask:
        # co-task every 10 ms needing half the CUs for 1 ms during a long launch
        per_root_ms = ms_c / len(timed)
        cus = rt.info["compute_units"]

        def cotask_run(opts, groups, seconds):
            k = max(1, int(seconds * 1e3 / max(per_root_ms, 1e-3)))
            k = min(k, 400000)
            d_many = rt._roots(np.resize(np.asarray(timed, dtype=np.uint32), k))
            h = coop.coop_bfs(rt.rt, dg.handle, d_many, k, level, 0, opts, stream)
            coop.coop_injector_start(rt.rt, h, groups=groups, busy_ns=1_000_000, period_ns=10_000_000)
            rc, st = coop.coop_wait(h)
            irc, cst = coop.coop_injector_stop(rt.rt)
            if rc != 0 or irc != 0:
                raise RuntimeError(f"co-task run failed: {coop.coop_strerror(rc)} / {coop.coop_strerror(irc)}")
            return d_many, st, cst

        d_many, st_m, cst = cotask_run(coop_opts, cus // 2, args.cotask_seconds)
        alone = run(coop_opts, d_many)
        result["cotask"] = {
            "period_ms": 10, "busy_ms": 1, "groups": cus // 2, "count": cst["count"],
            "latency_p50_ms": round(cst["latency_p50_ms"], 4), "latency_p99_ms": round(cst["latency_p99_ms"], 4),
            "latency_max_ms": round(cst["latency_max_ms"], 4),
            "gather_p50_ms": round(cst["gather_p50_ms"], 4), "gather_p99_ms": round(cst["gather_p99_ms"], 4),
            "busy_mean_ms": round(cst["busy_mean_ms"], 4),
            "traversal_ms_alone": round(alone["kernel_ms"], 2), "traversal_ms_with_cotask": round(st_m["kernel_ms"], 2),
            "slowdown": round(st_m["kernel_ms"] / alone["kernel_ms"], 4),
            "kills": st_m["kills"], "forks": st_m["forks"], "join_full": st_m["join_full"],
            "model_kernel_preemption": round(10 / 9, 4), "model_half_cu": round(10 / 9.5, 4),
        }
        log(f"cotask: {result['cotask']}")

        # gather time against the number of workgroups the co-task claims,
        # for the query barrier and the regular barrier (one kill per
        # barrier), as in the paper's responsiveness experiment
        regular_opts = coop.make_opts(coop.COOP_MODE_COOP,
                                      flags=coop.COOP_F_HOST_SCHEDULE | coop.COOP_F_REGULAR_BARRIER)
        sweep = []
        for groups in (1, cus // 4, cus // 2, cus - 1):
            for name, o in (("query", coop_opts), ("regular", regular_opts)):
                _, st_g, c_g = cotask_run(o, groups, args.gather_seconds)
                sweep.append({"groups": groups, "barrier": name, "count": c_g["count"],
                              "gather_p50_ms": round(c_g["gather_p50_ms"], 4),
                              "gather_p99_ms": round(c_g["gather_p99_ms"], 4),
                              "latency_p50_ms": round(c_g["latency_p50_ms"], 4),
                              "kills": st_g["kills"], "forks": st_g["forks"], "join_full": st_g["join_full"]})
        result["gather_sweep"] = sweep
        log("gather sweep: " + "; ".join(f"{e['barrier']} W={e['groups']}: {e['gather_p50_ms']}/{e['gather_p99_ms']} ms "
                                         f"({e['count']} co-tasks, {e['kills']} kills)" for e in sweep))

    if not args.skip_share and not args.skip_sssp:
        # two cooperative launches at once: a long BFS (R-MAT, ~0.3 s) and the
        # SSSP grid, equal weights; the sharer splits the resident workgroups
        per_root_ms = ms_c / len(timed)
        k = max(1, int(300.0 / max(per_root_ms, 1e-3)))
        d_many = rt._roots(np.resize(np.asarray(timed, dtype=np.uint32), k))
        st_a = run(coop_opts, d_many)
        st_b = run_s(coop_opts)
        s2 = torch.cuda.Stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coop.coop_share_start(rt.rt, 100)
        try:
            ha = coop.coop_bfs(rt.rt, dg.handle, d_many, k, level, 0, coop_opts, stream)
            coop.coop_share_add(rt.rt, ha, 1)
            hb = coop.coop_sssp(rt.rt, dgs.handle, d0, 1, dist, 0, coop_opts, s2)
            coop.coop_share_add(rt.rt, hb, 1)
            rcb, sh_b = coop.coop_wait(hb)
            rca, sh_a = coop.coop_wait(ha)
        finally:
            rcs, sst = coop.coop_share_stop(rt.rt)
        wall = (time.perf_counter() - t0) * 1e3
        if rca or rcb or rcs:
            raise RuntimeError(f"shared run failed: {rca} {rcb} {rcs}")
        result["shared"] = {
            "bfs_ms_alone": round(st_a["kernel_ms"], 2), "sssp_ms_alone": round(st_b["kernel_ms"], 2),
            "bfs_ms_shared": round(sh_a["kernel_ms"], 2), "sssp_ms_shared": round(sh_b["kernel_ms"], 2),
            "wall_ms_shared": round(wall, 2),
            "sequential_ms": round(st_a["kernel_ms"] + st_b["kernel_ms"], 2),
            "bfs_min_groups": sh_a["min_groups"], "sssp_max_groups": sh_b["max_groups"],
            "target_updates": sst["target_updates"],
        }
        log(f"shared: {result['shared']}")

    if not args.skip_octree:
        # work-stealing octree: 4M clustered points, leaves of at most 8
        xo, yo, zo = gg.points(4_000_000, 9, "clustered")
        no = len(xo)
        dxo, dyo, dzo = (torch.from_numpy(v.view(np.int32)).cuda() for v in (xo, yo, zo))
        o_out = torch.empty((no, 4), dtype=torch.int32, device="cuda")
        o_leaves = torch.empty((no, 8), dtype=torch.int32, device="cuda")

        def run_o(opts):
            h = coop.coop_octree(rt.rt, dxo, dyo, dzo, no, 8, o_out, o_leaves, no, opts, stream)
            rc, st = coop.coop_wait(h)
            if rc != 0:
                raise RuntimeError(coop.coop_strerror(rc))
            return st

        run_o(coop_opts)
        run_o(plain_opts)
        oc = [run_o(coop_opts) for _ in range(5)]
        op = [run_o(plain_opts) for _ in range(5)]
        ms_oc = float(np.median([s["kernel_ms"] for s in oc]))
        ms_op = float(np.median([s["kernel_ms"] for s in op]))
        # co-tasks needing half the CUs every 2 ms during one build
        h = coop.coop_octree(rt.rt, dxo, dyo, dzo, no, 8, o_out, o_leaves, no, coop_opts, stream)
        coop.coop_injector_start(rt.rt, h, groups=rt.info["compute_units"] // 2, busy_ns=200_000,
                                 period_ns=2_000_000)
        rc, st_oi = coop.coop_wait(h)
        irc, c_oi = coop.coop_injector_stop(rt.rt)
        if rc or irc:
            raise RuntimeError(f"octree co-task run failed: {rc} {irc}")
        result["octree"] = {
            "workload": "work-stealing octree, 4M clustered points (seed 9), leaves of at most 8 points",
            "ms_coop": round(ms_oc, 3), "ms_plain": round(ms_op, 3), "coop_overhead": round(ms_oc / ms_op, 4),
            "mpoints_per_s_coop": round(no / (ms_oc * 1e-3) / 1e6, 1),
            "splits": oc[0]["levels"], "leaves": oc[0]["rows"], "steals": oc[0]["arcs"],
            "cotask": {"period_ms": 2, "busy_ms": 0.2, "count": c_oi["count"],
                       "latency_p50_ms": round(c_oi["latency_p50_ms"], 4),
                       "latency_p99_ms": round(c_oi["latency_p99_ms"], 4),
                       "build_ms": round(st_oi["kernel_ms"], 3), "kills": st_oi["kills"]},
        }
        log(f"octree: {result['octree']}")

    if not args.skip_barrier:
        # global-barrier latency (persistent launch doing barriers only)
        bar = {}
        modes = (("plain", plain_opts),) if args.barrier_bench_plain else ()
        for name, o in modes + (("coop", coop_opts),):
            ns, _ = coop.coop_barrier_bench(rt.rt, 2000, o, stream)
            bar[name] = round(ns, 1)
        result["barrier_ns"] = bar
        log(f"barrier ns: {bar}")

    if args.copy_probe_mib > 0:
        x = torch.zeros(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda")
        y = x + 1
        torch.cuda.synchronize()
        del x, y

    traffic = committed_traffic()
    result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(achieved / HBM_PEAK_GBS, 4),
                          "traffic": None if traffic is None else int(traffic),
                          "kernel": "bfs_kernel<true>", "launch_ms": round(launch_ms, 4),
                          "alg_bytes_per_launch": int(alg_bytes_launch),
                          "kernel_counted_bytes_per_launch": int(counted),
                          "source_hash": kernel_source_hash()}

    # CPU baseline: the oracle (single-threaded FIFO BFS) on a bounded sample
    import oracle
    sample = timed[:args.cpu_sample]
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
