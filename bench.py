#!/usr/bin/env python3
"""Benchmark: cooperative vs plain persistent BFS on R-MAT scale 22 (the
headline), with the other measured configurations as side lines.

Headline workload (one GPU, the timed region and nothing else): R-MAT scale
22, edge factor 16 (a=0.57, b=0.19, c=0.19, d=0.05), seeded, permuted,
symmetrised, loops/duplicates removed, uint32 CSR resident in HBM. A *step*
is one BFS traversal from the next seeded source (degree >= 1). The K timed
steps run in ceil(K / L) persistent cooperative launches of L sources each
(the last one holds the remainder); at every resizing barrier the launch
queries the host-written scheduler target, which stays at N, so nothing is
killed or forked in the timed region. Warm-up runs ceil(W / L) launches of
L other sources. All timed launches are queued on the stream before the
first is waited for; the region is bracketed by torch.cuda.synchronize().

Printed JSON line (one):
  value          GTEPS of the cooperative launches: sum over the timed
                 sources of the undirected edges in the source's component
                 / wall time of the timed region
  plain          the same sources in plain persistent launches (fixed M)
  coop_overhead  cooperative / plain kernel time (HIP events)
  roofline       the BFS kernel: algorithmic bytes per launch (8 B per
                 scanned arc + 20 B per reached vertex) / mean launch time
                 vs 8 TB/s ("frac"); "traffic" = HBM bytes per launch from
                 the committed PMC summary when it was taken on the current
                 kernel sources and launch size, "traffic_frac" = that over
                 the launch time vs 8 TB/s
  er4096         ER n=4096, d=8: BFS from vertex 0, coop vs plain (median)
  sssp           frontier Bellman-Ford on the 1024x1024 grid: coop vs plain,
                 and 16 seeded random kill/fork schedules checked equal to
                 the never-resizing run
  cotask         a co-task every 10 ms needing half the CUs for 1 ms during
                 one long cooperative launch (>= 1000 samples): latency,
                 gather time, slowdown against the same launch alone
  gather_sweep   gather time against the workgroups a co-task claims, query
                 barrier vs the regular barrier
  shared         a long BFS and the SSSP grid launched together
  octree         work-stealing octree build, coop vs plain, with co-tasks
  batch          512 ER instances, BFS (+ colouring) in one launch: default
                 vs autotuned schedule
  barrier_ns     2000 barriers of an empty launch, cooperative and plain
  cpu_baseline   the oracle (one core) on a bounded sample of the headline
                 sources; all_cores: the OpenMP level-synchronous BFS
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
# the kernel, the runtime that sizes and parameterises its launches, and the
# graph preparation that orders the arcs its bottom-up levels probe
KERNEL_SOURCES = ("paper_1707_01989_amd/csrc/coop_kernels.hip", "paper_1707_01989_amd/csrc/traverse.h",
                  "paper_1707_01989_amd/csrc/coop_internal.h", "include/coop_device.hpp",
                  "paper_1707_01989_amd/csrc/coop_runtime.hip", "paper_1707_01989_amd/csrc/graph_prep.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(roots_per_launch: int):
    """HBM bytes per launch from the committed PMC summary, or None when the
    summary is missing, was taken on other kernel sources, or on launches of
    another size."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"^source_hash:\s*(\w+)", text, re.M)
    b = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    L = re.search(r"^roots_per_launch:\s*(\d+)", text, re.M)
    if not m or not b or not L or m.group(1) != kernel_source_hash() or int(L.group(1)) != roots_per_launch:
        return None
    return float(b.group(1))


def chunks(seq, L):
    return [seq[i:i + L] for i in range(0, len(seq), L)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="timed BFS sources (any count >= 1)")
    ap.add_argument("--warmup", type=int, default=10, help="warm-up sources (any count >= 0)")
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--roots-per-launch", type=int, default=10)
    ap.add_argument("--er-reps", type=int, default=21)
    ap.add_argument("--sssp-reps", type=int, default=11)
    ap.add_argument("--sssp-seeds", type=int, default=16)
    ap.add_argument("--cotask-seconds", type=float, default=10.5)
    ap.add_argument("--gather-seconds", type=float, default=0.5, help="per point of the gather-time sweep")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="bound on the oracle timing")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one int32 'x + 1' elementwise kernel over this many MiB (counter calibration)")
    for leg in ("er", "sssp", "cotask", "share", "octree", "batch", "barrier", "cpu"):
        ap.add_argument(f"--skip-{leg}", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; runs on several GPUs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        sys.exit("--steps must be >= 1 and --warmup >= 0")
    L = max(1, args.roots_per_launch)
    t_all = time.time()

    import numpy as np
    import torch

    from paper_1707_01989_amd import coop, graphgen as gg

    t0 = time.time()
    g = gg.rmat(args.scale, 16, seed=3)
    log(f"rmat{args.scale}: n={g.n} arcs={g.arcs} generated in {time.time() - t0:.1f}s")
    deg = g.degrees()
    n_warm = -(-args.warmup // L) * L if args.warmup else 0
    roots = gg.sources(g, 3, n_warm + args.steps)

    # per-source traversal sizes (component of each source)
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    A = csr_matrix((np.ones(g.arcs, dtype=np.int8), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                   shape=(g.n, g.n))
    _, comp = connected_components(A, directed=False)
    del A
    comp_edges = np.bincount(comp, weights=deg, minlength=comp.max() + 1) / 2
    comp_verts = np.bincount(comp, minlength=comp.max() + 1)
    edges_of = lambda r: float(comp_edges[comp[r]])
    verts_of = lambda r: int(comp_verts[comp[r]])

    rt = coop.Runtime(0)
    dg = rt.graph(g)
    timed = [int(r) for r in roots[n_warm:]]
    batches_w = [rt._roots(b) for b in chunks([int(r) for r in roots[:n_warm]], L)]
    batches_t = [rt._roots(b) for b in chunks(timed, L)]
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
        f"{len(sts_c)} launches, mean {launch_ms:.3f} ms, levels {sum(s['levels'] for s in sts_c)}")

    edges = sum(edges_of(r) for r in timed)
    verts = sum(verts_of(r) for r in timed)
    gteps_c = edges / wall_c / 1e9
    gteps_p = edges / wall_p / 1e9

    # algorithmic bytes of a level-synchronous BFS, at the data's natural
    # width: 8 B per scanned arc (column index + state probe) and 20 B per
    # reached vertex (row range, frontier read and write, level write);
    # arcs scanned = the degree sum of the reached vertices. Per launch =
    # the timed total over the timed launches (all of L sources unless the
    # step count is not a multiple of L).
    alg_bytes_launch = (8 * 2 * edges + 20 * verts) / len(sts_c)
    achieved = alg_bytes_launch / (launch_ms * 1e-3) / 1e9
    # what this kernel itself read, by its own counters (direction-optimising
    # BFS skips arcs): 4 B per arc examined, 8 B per row range, 4 B per
    # bitmap word
    counted = sum(4 * s["arcs"] + 8 * s["rows"] + 4 * s["bitmap_words"] for s in sts_c) / len(sts_c)
    uniform = args.steps % L == 0

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
                               f"one seeded source per step, {L} sources per persistent cooperative launch "
                               f"(scheduler target queried at every barrier and kept at N: no kill/fork, "
                               f"no co-task in the timed region)",
                   "n": g.n, "arcs": g.arcs, "sources": len(timed), "launches": len(sts_c),
                   "roots_per_launch": L, "groups": sts_c[0]["grid"], "group_size": 1024,
                   "warmup_sources_run": n_warm},
        "plain": {"value": round(gteps_p, 3), "kernel_ms": round(ms_p, 3), "wall_ms": round(wall_p * 1e3, 3)},
        "coop_overhead": round(ms_c / ms_p, 4),
        "kernel_ms": round(ms_c, 3),
        "wall_ms": round(wall_c * 1e3, 3),
        "barriers": sum(s["barriers"] for s in sts_c),
    }

    if not args.skip_er:
        # configuration 0: ER n = 4096, average degree 8 (seed 1), BFS from
        # vertex 0, one launch per run; latency bound (a handful of levels)
        ge = gg.er(4096, 8, 1)
        dge = rt.graph(ge)
        lv_e = torch.empty(ge.n, dtype=torch.int32, device="cuda")
        r0 = rt._roots([0])
        Ae = csr_matrix((np.ones(ge.arcs, dtype=np.int8), ge.col.astype(np.int64), ge.row_ptr.astype(np.int64)),
                        shape=(ge.n, ge.n))
        _, ce = connected_components(Ae, directed=False)
        e_edges = float(ge.degrees()[ce == ce[0]].sum() / 2)

        def run_e(opts):
            h = coop.coop_bfs(rt.rt, dge.handle, r0, 1, lv_e, 0, opts, stream)
            rc, st = coop.coop_wait(h)
            if rc != 0:
                raise RuntimeError(coop.coop_strerror(rc))
            return st

        def er_pair(flags):
            oc = coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_HOST_SCHEDULE | flags)
            op = coop.make_opts(coop.COOP_MODE_PLAIN, flags=flags)
            for _ in range(3):
                run_e(oc)
                run_e(op)
            ec, ep = [], []
            for _ in range(args.er_reps):            # interleaved, so drift hits both alike
                ec.append(run_e(oc))
                ep.append(run_e(op))
            mc = float(np.median([s["kernel_ms"] for s in ec]))
            mp = float(np.median([s["kernel_ms"] for s in ep]))
            dc = float(np.median([s["device_ms"] for s in ec]))
            dp = float(np.median([s["device_ms"] for s in ep]))
            return {
                "levels": ec[0]["levels"], "barriers": ec[0]["barriers"],
                "ms_coop": round(mc, 4), "ms_plain": round(mp, 4), "coop_overhead": round(mc / mp, 4),
                "gteps_coop": round(e_edges / (mc * 1e-3) / 1e9, 4),
                "gteps_plain": round(e_edges / (mp * 1e-3) / 1e9, 4),
                "ns_per_barrier_coop": round(dc * 1e6 / ec[0]["barriers"], 1),
                "ns_per_barrier_plain": round(dp * 1e6 / ep[0]["barriers"], 1),
            }
        # the configuration as stated: a global barrier after every level
        result["er4096"] = {
            "workload": "BFS from vertex 0, ER G(n=4096, m=16384) (seed 1), one persistent launch per run, "
                        "every level a phase of all workgroups followed by a global barrier",
            "reps": args.er_reps, **er_pair(coop.COOP_F_LEVEL_BARRIERS),
            "note": "ns per barrier = device time from the first barrier on / barriers (one level's work plus its barrier)",
            # the library's default: the master step runs small top-down levels itself
            "master_step_levels": er_pair(0),
        }
        log(f"er4096: {result['er4096']}")
        dge.release()

    if not args.skip_sssp:
        # configuration 1: frontier Bellman-Ford on the 1024x1024 grid,
        # w U[1,1000] (seed 2), source 0
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
        sc, sp = [], []
        for _ in range(args.sssp_reps):
            sc.append(run_s(coop_opts)["kernel_ms"])
            sp.append(run_s(plain_opts)["kernel_ms"])
        st_1 = run_s(coop_opts)
        ref = dist.clone()
        sched = []
        for seed in range(1, args.sssp_seeds + 1):
            rnd = coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_RANDOM_SCHEDULE | coop.COOP_F_PARK_KILLED,
                                 sched_seed=seed, sched_p=0.25)
            st_r = run_s(rnd)
            sched.append({"seed": seed, "ms": round(st_r["kernel_ms"], 3), "kills": st_r["kills"],
                          "forks": st_r["forks"], "min_groups": st_r["min_groups"],
                          "same_as_never_resize": bool(torch.equal(ref, dist))})
        e_s = gs.edges
        result["sssp"] = {
            "workload": "frontier Bellman-Ford, 1024x1024 grid, w U[1,1000] (seed 2), source 0",
            "reps": args.sssp_reps,
            "gteps_coop": round(e_s / (np.median(sc) * 1e-3) / 1e9, 4),
            "gteps_plain": round(e_s / (np.median(sp) * 1e-3) / 1e9, 4),
            "ms_coop": round(float(np.median(sc)), 3), "ms_plain": round(float(np.median(sp)), 3),
            "coop_overhead": round(float(np.median(sc) / np.median(sp)), 4),
            "rounds": st_1["barriers"],
            "ns_per_round_coop": round(float(np.median(sc)) * 1e6 / st_1["barriers"], 1),
            "random_schedules": {"p": 0.25, "seeds": len(sched),
                                 "all_same_as_never_resize": all(s["same_as_never_resize"] for s in sched),
                                 "kills": sum(s["kills"] for s in sched), "forks": sum(s["forks"] for s in sched),
                                 "ms_median": round(float(np.median([s["ms"] for s in sched])), 3),
                                 "runs": sched},
        }
        log(f"sssp: coop {result['sssp']['ms_coop']} ms plain {result['sssp']['ms_plain']} ms "
            f"ratio {result['sssp']['coop_overhead']}; schedules same: "
            f"{result['sssp']['random_schedules']['all_same_as_never_resize']}")

    if not args.skip_cotask:
        # configuration 2's co-task: every 10 ms, half the CUs for 1 ms, during
        # one long cooperative launch over the headline's sources
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
            "seconds": round(st_m["kernel_ms"] / 1e3, 2),
            "latency_p50_ms": round(cst["latency_p50_ms"], 4), "latency_p99_ms": round(cst["latency_p99_ms"], 4),
            "latency_max_ms": round(cst["latency_max_ms"], 4),
            "gather_p50_ms": round(cst["gather_p50_ms"], 4), "gather_p99_ms": round(cst["gather_p99_ms"], 4),
            "busy_mean_ms": round(cst["busy_mean_ms"], 4),
            "traversal_ms_alone": round(alone["kernel_ms"], 2), "traversal_ms_with_cotask": round(st_m["kernel_ms"], 2),
            "slowdown": round(st_m["kernel_ms"] / alone["kernel_ms"], 4),
            "gteps_with_cotask": round(sum(edges_of(int(r)) for r in d_many.cpu().numpy()) /
                                       (st_m["kernel_ms"] * 1e-3) / 1e9, 3),
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
        del dxo, dyo, dzo, o_out, o_leaves

    if not args.skip_batch:
        result["batch"] = batch_leg(rt, coop, gg, np, torch, stream)

    if not args.skip_barrier:
        # global-barrier latency (persistent launch doing barriers only)
        ns, _ = coop.coop_barrier_bench(rt.rt, 2000, coop_opts, stream)
        ns_p, _ = coop.coop_barrier_bench(rt.rt, 2000, plain_opts, stream)
        result["barrier_ns"] = {"coop": round(ns, 1), "plain": round(ns_p, 1),
                                "coop_overhead": round(ns / ns_p, 4)}
        log(f"barrier ns: {result['barrier_ns']}")

    if args.copy_probe_mib > 0:
        x = torch.zeros(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda")
        y = x + 1
        torch.cuda.synchronize()
        del x, y

    traffic = committed_traffic(L) if uniform else None
    result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(achieved / HBM_PEAK_GBS, 4),
                          "traffic": None if traffic is None else int(traffic),
                          "traffic_frac": None if traffic is None else
                          round(traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "frac_basis": "algorithmic bytes (8 B per arc of the reached vertices + 20 B per "
                                        "reached vertex) per launch / mean launch time",
                          "kernel": "bfs_kernel<true>", "launch_ms": round(launch_ms, 4),
                          "units_per_launch": L if uniform else round(len(timed) / len(sts_c), 3),
                          "alg_bytes_per_launch": int(alg_bytes_launch),
                          "kernel_counted_bytes_per_launch": int(counted),
                          "source_hash": kernel_source_hash()}

    if not args.skip_cpu:
        result["cpu_baseline"] = cpu_leg(g, timed, edges_of, args.cpu_seconds)
    rt.close()
    result["bench_wall_s"] = round(time.time() - t_all, 1)
    print(json.dumps(result), flush=True)


def batch_leg(rt, coop, gg, np, torch, stream):
    """Configuration 3: 512 ER instances (n log-uniform in [2^10, 2^18),
    average degree U[4, 32], seeds 1000 + i), BFS from vertex 0 (then greedy
    colouring with priority seed i) per instance in one launch; the default
    schedule against the autotuned one (median of 3 launches each)."""
    t0 = time.time()
    gs = gg.er_batch(512, 1000, workers=16)
    dgs = [rt.graph(g) for g in gs]
    log(f"batch: 512 instances, n={sum(g.n for g in gs)} arcs={sum(g.arcs for g in gs)} "
        f"({time.time() - t0:.1f}s)")
    copts = coop.make_opts(coop.COOP_MODE_COOP)
    out = {"workload": "512 ER instances, n = floor(2^U(10,18)), d = U(4,32), seeds 1000+i; "
                       "BFS from vertex 0 (+ greedy colouring, priority seed i) per instance, one launch",
           "instances": len(gs), "n_total": int(sum(g.n for g in gs)), "arcs_total": int(sum(g.arcs for g in gs))}
    bfs_edges = None
    for name, ops in (("bfs", coop.COOP_BATCH_BFS), ("bfs_color", coop.COOP_BATCH_BFS | coop.COOP_BATCH_COLOR)):
        items, outs = rt.batch_items(dgs, ops)
        rt.batch(items, None, copts)             # warm-up
        if bfs_edges is None:
            torch.cuda.synchronize()
            bfs_edges = 0.0
            for g, o in zip(gs, outs):
                reached = o["level"].cpu().numpy().view(np.uint32) != 0xFFFFFFFF
                bfs_edges += float(g.degrees()[reached].sum()) / 2
        ta = time.time()
        best, best_ms, def_ms = coop.coop_batch_autotune(rt.rt, items, stride=1, reps=3, opts=copts)
        tune_s = time.time() - ta
        res = {}
        for tname, tune in (("default", None), ("tuned", best)):
            ms = []
            for _ in range(3):
                rc, st = rt.batch(items, tune, copts)
                if rc != 0:
                    raise RuntimeError(coop.coop_strerror(rc))
                ms.append(st["kernel_ms"])
            res[tname] = float(np.median(ms))
        out[name] = {"ms_default": round(res["default"], 3), "ms_tuned": round(res["tuned"], 3),
                     "speedup_tuned": round(res["default"] / res["tuned"], 4),
                     "tuned": best.as_dict(), "tune_seconds": round(tune_s, 1),
                     "search_ms_default": round(def_ms, 3) if def_ms > 0 else None,
                     "search_ms_tuned": round(best_ms, 3)}
        if name == "bfs":
            out[name]["gteps_default"] = round(bfs_edges / (res["default"] * 1e-3) / 1e9, 3)
            out[name]["gteps_tuned"] = round(bfs_edges / (res["tuned"] * 1e-3) / 1e9, 3)
        log(f"batch {name}: {out[name]}")
        del items, outs
    for dg in dgs:
        dg.release()
    return out


def cpu_leg(g, timed, edges_of, seconds):
    """The oracle's FIFO BFS on one core, over as many of the timed sources
    as fit in `seconds` (at least one); then the OpenMP level-synchronous
    BFS on every host core over the same sources."""
    import oracle
    sample = []
    t = time.perf_counter()
    for r in timed:
        oracle.bfs(g, r)
        sample.append(r)
        if time.perf_counter() - t >= seconds:
            break
    cpu_s = time.perf_counter() - t
    cpu_edges = sum(edges_of(r) for r in sample)
    t = time.perf_counter()
    used = 0
    for r in sample:
        _, used = oracle.bfs_parallel(g, r)
    par_s = time.perf_counter() - t
    res = {"value": round(cpu_edges / cpu_s / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
           "sample": f"{len(sample)} of the timed sources of the same graph, {cpu_s:.2f} s",
           "all_cores": {"value": round(cpu_edges / par_s / 1e9, 5), "unit": "GTEPS", "cores": used,
                         "nproc": os.cpu_count(), "kind": "OpenMP level-synchronous BFS",
                         "sample": f"the same {len(sample)} sources, {par_s:.2f} s"}}
    log(f"cpu: {res}")
    return res


if __name__ == "__main__":
    main()
