"""GPU parity: every HIP path against the CPU oracle, element by element.

All results are integers with a unique correct value, so the bar is bit
equality, under plain launches, cooperative launches, and cooperative
launches under seeded kill/fork schedules (any schedule must give the
never-resizing schedule's result)."""
import sys
import time

import numpy as np
import pytest

import oracle
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rt():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1707_01989_amd import coop
    r = coop.Runtime(0)
    say(f"device: {r.info}")
    yield r
    r.close()


@pytest.fixture(scope="module")
def coop_mod():
    from paper_1707_01989_amd import coop
    return coop


def as_u32(t):
    return t.cpu().numpy().view(np.uint32)


def check_rows(out, roots, g):
    """Every traversal's own output row (out_stride = n) equals the oracle's
    levels for its source: the traversals that ran while workgroups were
    being killed and forked are checked, not only the last one."""
    got = out.cpu().numpy().view(np.uint32).reshape(len(roots), g.n)
    exp = {}
    for i, r in enumerate(roots):
        r = int(r)
        if r not in exp:
            exp[r] = oracle.bfs(g, r)
        assert np.array_equal(got[i], exp[r]), f"traversal {i} (source {r})"


def modes(coop):
    return {
        "plain": coop.make_opts(coop.COOP_MODE_PLAIN),
        "coop": coop.make_opts(coop.COOP_MODE_COOP),
        "coop_host": coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_HOST_SCHEDULE),
        "coop_topdown": coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_TOP_DOWN_ONLY),
        "coop_levels": coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_LEVEL_BARRIERS),
        # BFS level counts from the statistics slots, not the barrier arrivals
        "coop_slot_sums": coop.make_opts(coop.COOP_MODE_COOP, flags=coop.COOP_F_SLOT_SUMS),
        "plain_slot_sums": coop.make_opts(coop.COOP_MODE_PLAIN, flags=coop.COOP_F_SLOT_SUMS),
    }


# ------------------------------------------------------------------ BFS

@pytest.mark.parametrize("mode", ["plain", "coop", "coop_host", "coop_topdown"])
def test_bfs_er4096(rt, coop_mod, gg, mode):
    g = gg.er(4096, 8, 1)
    say(f"bfs er4096 mode={mode}")
    dg = rt.graph(g)
    rc, lv, st = rt.bfs(dg, [0], modes(coop_mod)[mode])
    assert rc == 0, coop_mod.coop_strerror(rc)
    assert np.array_equal(as_u32(lv), oracle.bfs(g, 0))
    assert st["kills"] == 0
    dg.release()


@pytest.mark.parametrize("name", ["path", "star_leaf", "disjoint", "isolated", "cycle", "grid", "tree"])
def test_bfs_small_graphs(rt, coop_mod, gg, name):
    g, src = {
        "path": (gg.path(300), 7),
        "star_leaf": (gg.star(200), 5),
        "disjoint": (gg.disjoint_union(gg.cycle(50), gg.path(40)), 60),
        "isolated": (gg.disjoint_union(gg.empty(3), gg.path(5)), 1),
        "cycle": (gg.cycle(1001), 0),
        "grid": (gg.grid(17, 23), 40),
        "tree": (gg.binary_tree(2047), 0),
    }[name]
    say(f"bfs small {name}")
    dg = rt.graph(g)
    exp = oracle.bfs(g, src)
    for mode, o in modes(coop_mod).items():
        rc, lv, _ = rt.bfs(dg, [src], o)
        assert rc == 0, (mode, coop_mod.coop_strerror(rc))
        assert np.array_equal(as_u32(lv), exp), mode
    dg.release()


@pytest.mark.parametrize("th,strip", [(128, 4096), (16, 64), (4, 8)])
def test_bfs_rmat_heavy_strips(rt, coop_mod, gg, th, strip):
    g = gg.rmat(14, 16, seed=3)
    src = int(gg.sources(g, 1, 1)[0])
    say(f"bfs rmat14 heavy_th={th} strip={strip}")
    dg = rt.graph(g)
    exp = oracle.bfs(g, src)
    for mode in ("plain", "coop", "coop_topdown"):
        o = modes(coop_mod)[mode]
        o.heavy_threshold = th
        o.strip = strip
        rc, lv, st = rt.bfs(dg, [src], o)
        assert rc == 0, coop_mod.coop_strerror(rc)
        assert np.array_equal(as_u32(lv), exp), mode
        say(f"  {mode}: td={st['td_levels']} bu={st['bu_levels']} heavy={st['heavy_phases']} arcs={st['arcs']}")
    dg.release()


@pytest.mark.parametrize("name", ["path", "tree", "er4096", "grid", "rmat14", "rmat16"])
def test_bfs_master_step_levels(rt, coop_mod, gg, name):
    """Small top-down levels run by the master step give the levels of the
    launch that gives every level its own phase and barrier, for every
    source, with the same level count and fewer barriers; narrow launches
    (small LDS lists, more workgroups than the master can gather) too."""
    c = coop_mod
    g = {"path": gg.path(3000), "tree": gg.binary_tree(4095), "er4096": gg.er(4096, 8, 1),
         "grid": gg.grid(40, 50), "rmat14": gg.rmat(14, 16, seed=3), "rmat16": gg.rmat(16, 16, seed=6)}[name]
    roots = gg.sources(g, 11, 6)
    say(f"bfs master-step levels {name} roots={roots.tolist()}")
    dg = rt.graph(g)
    for mode in (c.COOP_MODE_PLAIN, c.COOP_MODE_COOP):
        for ng, gs in ((0, 1024), (0, 256), (24, 64)):
            res = {}
            for flags in (0, c.COOP_F_LEVEL_BARRIERS):
                o = c.make_opts(mode, flags=flags, num_groups=ng, group_size=gs)
                rc, lv, st = rt.bfs(dg, roots, o)
                assert rc == 0, c.coop_strerror(rc)
                check_rows(lv.reshape(-1), roots, g)
                res[flags] = st
            a, b = res[0], res[c.COOP_F_LEVEL_BARRIERS]
            say(f"  mode={mode} groups={ng}x{gs}: levels {a['levels']} / {b['levels']}, "
                f"barriers {a['barriers']} / {b['barriers']}")
            assert a["levels"] == b["levels"]
            assert a["barriers"] <= b["barriers"]
    dg.release()


def test_bfs_multi_root(rt, coop_mod, gg):
    g = gg.rmat(13, 16, seed=5)
    roots = gg.sources(g, 2, 6)
    say(f"bfs multi-root rmat13 roots={roots.tolist()}")
    dg = rt.graph(g)
    for mode in ("plain", "coop", "coop_topdown", "coop_slot_sums"):
        rc, lv, st = rt.bfs(dg, roots, modes(coop_mod)[mode])
        assert rc == 0
        got = lv.cpu().numpy().view(np.uint32)
        for i, r in enumerate(roots):
            assert np.array_equal(got[i], oracle.bfs(g, int(r))), (mode, i)
    dg.release()


def test_bfs_small_groups(rt, coop_mod, gg):
    """Few and narrow workgroups: many claims per workgroup, ragged tails."""
    g = gg.er(20000, 6, 9)
    say("bfs er20000 narrow launches")
    dg = rt.graph(g)
    exp = oracle.bfs(g, 3)
    for mode in ("plain", "coop", "coop_topdown"):
        for ng, gs in ((1, 64), (3, 128), (7, 256), (40, 1024)):
            o = modes(coop_mod)[mode]
            o.num_groups = ng
            o.group_size = gs
            rc, lv, st = rt.bfs(dg, [3], o)
            assert rc == 0, (mode, ng, gs, coop_mod.coop_strerror(rc))
            assert np.array_equal(as_u32(lv), exp), (mode, ng, gs)
    dg.release()


@pytest.mark.parametrize("mode", ["plain", "coop"])
def test_source_outside_graph_fails_cleanly(rt, coop_mod, gg, mode):
    """A source >= n ends the launch with COOP_E_INVALID before anything is
    written for it (the kernel checks it before any access it indexes);
    the sources before it are complete and the runtime stays usable."""
    c = coop_mod
    g = gg.add_weights(gg.er(3000, 6, 4), 3, 1, 100)
    dg = rt.graph(g)
    o = modes(c)[mode]
    say(f"source outside the graph, {mode}: n={g.n}")
    for bad in (g.n, g.n + 40, 0xFFFFFFFF):
        rc, lv, _ = rt.bfs(dg, [5, bad], o)
        assert rc == c.COOP_E_INVALID, (bad, c.coop_strerror(rc))
        assert np.array_equal(lv[0].cpu().numpy().view(np.uint32), oracle.bfs(g, 5)), bad
        rc, d, _ = rt.sssp(dg, [7, bad], o)
        assert rc == c.COOP_E_INVALID, (bad, c.coop_strerror(rc))
        assert np.array_equal(d[0].cpu().numpy(), oracle.sssp(g, 7)), bad
    rc, lv, _ = rt.bfs(dg, [g.n - 1], o)
    assert rc == 0 and np.array_equal(as_u32(lv), oracle.bfs(g, g.n - 1))
    dg.release()


def test_graph_wrap_rejects_bad_csr(rt, coop_mod, gg):
    """coop_graph_wrap checks the CSR before any kernel indexes with it: a
    column index >= n (found by a device pass over the columns) or a bad
    row_ptr gives COOP_E_INVALID and no graph; the exact array is accepted."""
    import torch
    c = coop_mod
    g = gg.er(2000, 5, 6)
    rp = torch.from_numpy(g.row_ptr.view("int32")).cuda()
    col = g.col.copy()
    say(f"graph wrap checks: n={g.n} arcs={g.arcs}")
    h = c.coop_graph_wrap(rt.rt, rp, torch.from_numpy(col.view("int32")).cuda(), None, g.n, g.arcs)
    c.coop_graph_release(h)
    for pos, val in ((0, g.n), (g.arcs - 1, g.n + 7), (g.arcs // 2, 0xFFFFFFFF)):
        bad = col.copy()
        bad[pos] = val
        with pytest.raises(c.CoopError) as ei:
            c.coop_graph_wrap(rt.rt, rp, torch.from_numpy(bad.view("int32")).cuda(), None, g.n, g.arcs)
        assert ei.value.code == c.COOP_E_INVALID, (pos, val)
    dcol = torch.from_numpy(col.view("int32")).cuda()
    rp_bad = g.row_ptr.copy()
    rp_bad[10] = rp_bad[11] + 1                   # row 10 ends before it starts
    for r, arcs in ((rp_bad, g.arcs), (g.row_ptr, g.arcs - 1)):
        with pytest.raises(c.CoopError) as ei:
            c.coop_graph_wrap(rt.rt, torch.from_numpy(r.view("int32")).cuda(), dcol, None, g.n, arcs)
        assert ei.value.code == c.COOP_E_INVALID


def test_launch_limit(rt, coop_mod, gg):
    """N is at most 2048 (the launch context's per-id tables): 2049 is refused
    before any launch; a cooperative launch of exactly 2048 workgroups (far
    more than are resident at once: the rest start later as joiners or
    after the end) gives the oracle's levels."""
    c = coop_mod
    g = gg.er(3000, 5, 12)
    dg = rt.graph(g)
    say("launch limit: 2049 refused, 2048 coop")
    for mode in (c.COOP_MODE_PLAIN, c.COOP_MODE_COOP):
        o = c.make_opts(mode)
        o.num_groups = 2049
        with pytest.raises(c.CoopError) as ei:
            rt.bfs(dg, [1], o)
        assert ei.value.code == c.COOP_E_INVALID
    o = c.make_opts(c.COOP_MODE_COOP)
    o.num_groups = 2048
    o.group_size = 64
    rc, lv, st = rt.bfs(dg, [1], o)
    assert rc == 0, c.coop_strerror(rc)
    assert np.array_equal(as_u32(lv), oracle.bfs(g, 1))
    assert st["max_groups"] <= 2048
    dg.release()


def test_server_refuses_while_switched_off(rt, coop_mod, gg):
    """The query server is switched off until the cause of its GPU fault is
    shown: coop_server_create must refuse (COOP_E_INVALID) before it
    allocates or launches anything, not start a launch."""
    c = coop_mod
    dg = rt.graph(gg.add_weights(gg.er(500, 4, 3), 1, 1, 10))
    with pytest.raises(c.CoopError) as ei:
        c.coop_server_create(rt.rt, [dg.handle], 1 << 26, c.make_server_cfg())
    assert ei.value.code == c.COOP_E_INVALID
    dg.release()


# ----------------------------------------------------------------- SSSP

@pytest.mark.parametrize("name", ["grid64", "er5000", "rmat12"])
def test_sssp(rt, coop_mod, gg, name):
    g = {"grid64": lambda: gg.add_weights(gg.grid(64, 64), 2, 1, 1000),
         "er5000": lambda: gg.add_weights(gg.er(5000, 6, 4), 4, 1, 1000),
         "rmat12": lambda: gg.add_weights(gg.rmat(12, 16, seed=4), 4, 1, 255)}[name]()
    src = int(gg.sources(g, 6, 1)[0])
    say(f"sssp {name} src={src}")
    dg = rt.graph(g)
    exp = oracle.sssp(g, src)
    for mode, o in modes(coop_mod).items():
        o.heavy_threshold = 32
        o.strip = 128
        rc, d, st = rt.sssp(dg, [src], o)
        assert rc == 0, (mode, coop_mod.coop_strerror(rc))
        assert np.array_equal(d.cpu().numpy(), exp), mode
    dg.release()


def test_sssp_multi_root(rt, coop_mod, gg):
    g = gg.add_weights(gg.rmat(12, 16, seed=9), 3, 1, 255)
    roots = gg.sources(g, 4, 5)
    say(f"sssp multi-root rmat12 roots={roots.tolist()}")
    dg = rt.graph(g)
    for mode in ("plain", "coop"):
        rc, d, st = rt.sssp(dg, roots, modes(coop_mod)[mode])
        assert rc == 0, coop_mod.coop_strerror(rc)
        got = d.cpu().numpy()
        for i, r in enumerate(roots):
            assert np.array_equal(got[i], oracle.sssp(g, int(r))), (mode, i)
    dg.release()


def test_sssp_overflow_reported(rt, coop_mod, gg):
    g = gg.constant_weights(gg.path(6), 1_000_000_000)
    say("sssp overflow path")
    dg = rt.graph(g)
    rc, d, st = rt.sssp(dg, [0], modes(coop_mod)["coop"])
    assert rc == coop_mod.COOP_E_OVERFLOW
    dg.release()


@pytest.mark.parametrize("seed", range(8))
def test_sssp_random_schedule_park(rt, coop_mod, gg, seed):
    """Seeded kill/fork schedule (target redrawn at a quarter of the
    barriers); killed workgroups queue again as joiners."""
    g = gg.add_weights(gg.grid(96, 96), 2, 1, 1000)
    say(f"sssp grid96 random schedule seed={seed}")
    dg = rt.graph(g)
    exp = oracle.sssp(g, 0)
    o = coop_mod.make_opts(coop_mod.COOP_MODE_COOP,
                           flags=coop_mod.COOP_F_RANDOM_SCHEDULE | coop_mod.COOP_F_PARK_KILLED,
                           sched_seed=seed, sched_p=0.25, num_groups=32, group_size=256)
    rc, d, st = rt.sssp(dg, [0], o)
    assert rc == 0, coop_mod.coop_strerror(rc)
    assert np.array_equal(d.cpu().numpy(), exp)
    assert st["kills"] > 0 and st["forks"] > 0 and st["resizes"] > 0
    say(f"  rounds={st['levels']} kills={st['kills']} forks={st['forks']} M in [{st['min_groups']},{st['max_groups']}]")
    dg.release()


@pytest.mark.parametrize("seed", range(4))
def test_bfs_rmat_random_schedule(rt, coop_mod, gg, seed):
    """Direction-optimizing BFS under seeded kill/fork schedules (parked)."""
    g = gg.rmat(15, 16, seed=7)
    src = int(gg.sources(g, 5, 1)[0])
    say(f"bfs rmat15 random schedule seed={seed}")
    dg = rt.graph(g)
    exp = oracle.bfs(g, src)
    o = coop_mod.make_opts(coop_mod.COOP_MODE_COOP,
                           flags=coop_mod.COOP_F_RANDOM_SCHEDULE | coop_mod.COOP_F_PARK_KILLED,
                           sched_seed=100 + seed, sched_p=0.6, num_groups=64, group_size=256,
                           heavy_threshold=32, strip=256)
    rc, lv, st = rt.bfs(dg, [src], o)
    assert rc == 0, coop_mod.coop_strerror(rc)
    assert np.array_equal(as_u32(lv), exp)
    say(f"  td={st['td_levels']} bu={st['bu_levels']} kills={st['kills']} forks={st['forks']}")
    dg.release()


def test_bfs_random_schedule_with_joiner_grid(rt, coop_mod, gg):
    """Killed workgroups really exit; a separately launched joiner grid
    supplies the forks."""
    g = gg.grid(128, 128)
    say("bfs grid128 random schedule with joiner grid")
    dg = rt.graph(g)
    exp = oracle.bfs(g, 0)
    import torch
    roots = rt._roots([0])
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    o = coop_mod.make_opts(coop_mod.COOP_MODE_COOP, flags=coop_mod.COOP_F_RANDOM_SCHEDULE,
                           sched_seed=11, sched_p=0.3, num_groups=24, group_size=256)
    h = coop_mod.coop_bfs(rt.rt, dg.handle, roots, 1, out, 0, o)
    coop_mod.coop_fork_groups(h, 600)
    rc, st = coop_mod.coop_wait(h)
    assert rc == 0, coop_mod.coop_strerror(rc)
    assert np.array_equal(as_u32(out), exp)
    say(f"  kills={st['kills']} forks={st['forks']}")
    assert st["kills"] > 0
    dg.release()


# ------------------------------------------------------ colouring / MIS

# lanes per frontier vertex by average degree: grid 1, er8 2, er and rmat 4,
# rmat14 and complete 8 (complete(70) also needs colours past 64)
@pytest.mark.parametrize("name", ["er", "er8", "grid", "rmat", "rmat14", "complete", "empty"])
def test_color_and_mis(rt, coop_mod, gg, name):
    g = {"er": lambda: gg.er(6000, 16, 8), "er8": lambda: gg.er(5000, 8, 4), "grid": lambda: gg.grid(60, 70),
         "rmat": lambda: gg.rmat(12, 8, seed=2), "rmat14": lambda: gg.rmat(14, 16, seed=4),
         "complete": lambda: gg.complete(70), "empty": lambda: gg.empty(100)}[name]()
    say(f"color/mis {name}")
    dg = rt.graph(g)
    for seed in (0, 12345):
        ec = oracle.color(g, seed)
        em = oracle.mis(g, seed)
        for mode in ("plain", "coop"):
            o = modes(coop_mod)[mode]
            rc, c, _ = rt.color(dg, seed, o)
            assert rc == 0
            assert np.array_equal(as_u32(c), ec), (mode, seed)
            rc, m, _ = rt.mis(dg, seed, o)
            assert rc == 0
            assert np.array_equal(m.cpu().numpy(), em), (mode, seed)
    dg.release()


def test_color_random_schedule(rt, coop_mod, gg):
    g = gg.er(20000, 12, 21)
    say("color er20000 random schedule")
    dg = rt.graph(g)
    exp = oracle.color(g, 77)
    for seed in range(3):
        o = coop_mod.make_opts(coop_mod.COOP_MODE_COOP,
                               flags=coop_mod.COOP_F_RANDOM_SCHEDULE | coop_mod.COOP_F_PARK_KILLED,
                               sched_seed=seed, sched_p=0.5, num_groups=16, group_size=256)
        rc, c, st = rt.color(dg, 77, o)
        assert rc == 0
        assert np.array_equal(as_u32(c), exp), seed
    dg.release()


@pytest.mark.parametrize("seed", range(4))
def test_mis_random_schedule(rt, coop_mod, gg, seed):
    """Greedy MIS (the same priority DAG as colouring) under a seeded random
    kill/fork schedule: killed workgroups re-queue and are forked back in;
    the set equals the oracle's."""
    g = gg.er(20000, 12, 31) if seed % 2 == 0 else gg.rmat(14, 16, seed=5)
    say(f"mis {g.name} random schedule seed={seed}")
    dg = rt.graph(g)
    exp = oracle.mis(g, 99 + seed)
    o = coop_mod.make_opts(coop_mod.COOP_MODE_COOP,
                           flags=coop_mod.COOP_F_RANDOM_SCHEDULE | coop_mod.COOP_F_PARK_KILLED,
                           sched_seed=100 + seed, sched_p=0.5, num_groups=16, group_size=256)
    rc, m, st = rt.mis(dg, 99 + seed, o)
    say(f"  kills={st['kills']} forks={st['forks']} min={st['min_groups']}")
    assert rc == 0, coop_mod.coop_strerror(rc)
    assert np.array_equal(m.cpu().numpy(), exp)
    assert st["kills"] > 0
    dg.release()


# ---------------------------------------------------------- barrier

@pytest.mark.parametrize("mode", ["plain", "coop", "coop_host"])
def test_barrier_bench(rt, coop_mod, mode):
    say(f"barrier bench {mode}")
    ns, st = coop_mod.coop_barrier_bench(rt.rt, 2000, modes(coop_mod)[mode])
    say(f"  {ns:.0f} ns/barrier, grid={st['grid']} M={st['final_groups']}")
    assert st["barriers"] == 2001 and ns > 0
    assert st["final_groups"] == st["grid"]


@pytest.mark.parametrize("mode", ["plain", "coop"])
def test_barrier_watchdog_ends_a_launch_that_lost_a_workgroup(rt, coop_mod, mode):
    """A workgroup that goes missing (the last one leaves after the first
    barrier, made to from the host) must not hang the launch: every other
    workgroup's bounded wait runs out after the watchdog time, the launch
    ends with COOP_E_TIMEOUT, and the runtime goes on working."""
    c = coop_mod
    m = c.COOP_MODE_PLAIN if mode == "plain" else c.COOP_MODE_COOP
    o = c.make_opts(m, flags=c.COOP_F_TEST_LOSE_ONE, num_groups=16, group_size=256, watchdog_ns=50_000_000)
    say(f"barrier watchdog {mode}")
    t0 = time.time()
    with pytest.raises(c.CoopError) as ei:
        c.coop_barrier_bench(rt.rt, 100, o)
    took = time.time() - t0
    say(f"  {ei.value} after {took:.3f} s")
    assert ei.value.code == c.COOP_E_TIMEOUT
    assert took < 5.0
    ns, st = c.coop_barrier_bench(rt.rt, 50, c.make_opts(m, num_groups=16, group_size=256))
    assert st["barriers"] == 51 and st["error"] == 0


def test_plain_single_step_without_flags_in_lds(rt, coop_mod, gg):
    """Regression: kernels whose single barrier step keeps its flags outside
    the barrier's LDS block (connected components, the barrier benchmark),
    in plain launches, back to back, so that a workgroup's LDS still holds
    the previous launch's DONE flags when it masters the next launch's
    first barrier. Every launch must finish with the oracle's labels."""
    g = gg.rmat(14, 8, seed=1)
    exp = oracle.cc(g)
    dg = rt.graph(g)
    o = coop_mod.make_opts(coop_mod.COOP_MODE_PLAIN, watchdog_ns=2_000_000_000)
    for rep in range(12):
        rc, lab, st = rt.cc(dg, o)
        assert rc == 0, f"launch {rep}: {coop_mod.coop_strerror(rc)}"
        assert np.array_equal(lab.cpu().numpy().view(np.uint32), exp), f"launch {rep}"
        ns, bst = coop_mod.coop_barrier_bench(rt.rt, 50, o)
        assert bst["error"] == 0 and bst["barriers"] == 51, f"launch {rep}"
    dg.release()


# ------------------------------------------------- host target, co-tasks

def test_bfs_host_target_xcd_kills(rt, coop_mod, gg):
    """A host-driven target claims workgroups XCD by XCD (victims renumbered)
    while the kernel runs many sources; a joiner grid brings them back. Every
    source's levels equal the oracle's."""
    import time
    import torch
    c = coop_mod
    g = gg.rmat(16, 16, seed=9)
    say("bfs rmat16 host target with XCD-aware kills")
    dg = rt.graph(g)
    roots = [int(r) for r in gg.sources(g, 4, 24)]
    k = 400
    reps = np.resize(np.asarray(roots, dtype=np.uint32), k)
    d_roots = rt._roots(reps)
    out = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
    # the same 24 sources over and over: each output row is rewritten by identical runs
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    lv = torch.empty(k * g.n, dtype=torch.int32, device="cuda")
    h = c.coop_bfs(rt.rt, dg.handle, d_roots, k, lv, g.n, o)
    n = c.coop_handle_groups(h)
    for step in range(6):
        time.sleep(0.004)
        c.coop_set_target(h, n // 2 if step % 2 == 0 else n)
        if step % 2 == 1:
            c.coop_fork_groups(h, n // 2)
    rc, st = c.coop_wait(h)
    assert rc == 0, c.coop_strerror(rc)
    say(f"  kills={st['kills']} forks={st['forks']} min={st['min_groups']} ms={st['kernel_ms']:.1f}")
    assert st["kills"] > 0
    check_rows(lv, reps, g)
    # and a multi-root launch under the same schedule writes every row right
    d24 = rt._roots(roots)
    h = c.coop_bfs(rt.rt, dg.handle, d24, len(roots), out, g.n, o)
    c.coop_set_target(h, n // 3)
    time.sleep(0.002)
    c.coop_set_target(h, n)
    c.coop_fork_groups(h, n)
    rc, st = c.coop_wait(h)
    assert rc == 0, c.coop_strerror(rc)
    got = out.cpu().numpy().view(np.uint32).reshape(len(roots), g.n)
    for i, r in enumerate(roots):
        assert np.array_equal(got[i], oracle.bfs(g, r)), f"root {r}"
    dg.release()


def test_cotask_injector_during_bfs(rt, coop_mod, gg):
    """Co-tasks needing half the CUs run while a cooperative BFS holds the
    GPU: the kernel frees compute units on every shader engine (the hardware
    deals the co-task's workgroups round-robin over XCDs and their engines),
    so each co-task runs at once instead of waiting for the traversal."""
    import torch
    c = coop_mod
    g = gg.rmat(18, 16, seed=3)
    dg = rt.graph(g)
    roots = np.resize(gg.sources(g, 3, 16), 600).astype(np.uint32)
    d_roots = rt._roots(roots)
    lv = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    cus = rt.info["compute_units"]
    say("co-task injector during bfs rmat18")
    h = c.coop_bfs(rt.rt, dg.handle, d_roots, len(roots), lv, g.n, o)
    c.coop_injector_start(rt.rt, h, groups=cus // 2, busy_ns=500_000, period_ns=5_000_000)
    rc, st = c.coop_wait(h)
    irc, cst = c.coop_injector_stop(rt.rt)
    assert rc == 0 and irc == 0
    say(f"  kernel {st['kernel_ms']:.1f} ms kills={st['kills']} co-tasks={cst['count']} "
        f"p50={cst['latency_p50_ms']:.3f} p99={cst['latency_p99_ms']:.3f} max={cst['latency_max_ms']:.3f} ms")
    check_rows(lv, roots, g)
    assert cst["count"] >= 3
    # no co-task waited for the whole traversal
    assert cst["latency_max_ms"] < 0.5 * st["kernel_ms"]
    dg.release()


def test_regular_barrier_under_cotasks(rt, coop_mod, gg):
    """The regular resizing barrier (one workgroup leaves per barrier) gives
    the same levels under co-tasks; its gathers take more barriers than the
    query barrier's."""
    import torch
    c = coop_mod
    g = gg.rmat(18, 16, seed=3)
    dg = rt.graph(g)
    roots = np.resize(gg.sources(g, 3, 16), 300).astype(np.uint32)
    d_roots = rt._roots(roots)
    lv = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
    cus = rt.info["compute_units"]
    res = {}
    for name, extra in (("query", 0), ("regular", c.COOP_F_REGULAR_BARRIER)):
        o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE | extra)
        say(f"bfs rmat18 x{len(roots)} under co-tasks, {name} barrier")
        lv.fill_(-5)
        h = c.coop_bfs(rt.rt, dg.handle, d_roots, len(roots), lv, g.n, o)
        c.coop_injector_start(rt.rt, h, groups=cus // 4, busy_ns=300_000, period_ns=3_000_000)
        rc, st = c.coop_wait(h)
        irc, cst = c.coop_injector_stop(rt.rt)
        assert rc == 0 and irc == 0, (c.coop_strerror(rc), c.coop_strerror(irc))
        check_rows(lv, roots, g)
        say(f"  kernel {st['kernel_ms']:.1f} ms barriers={st['barriers']} kills={st['kills']} "
            f"co-tasks={cst['count']} gather p50={cst['gather_p50_ms']:.3f} ms")
        assert cst["count"] >= 1 and st["kills"] > 0
        res[name] = st
    # each co-task claims cus/4 workgroups: the regular barrier needs at
    # least that many kill barriers per co-task, the query barrier one
    assert res["regular"]["resizes"] >= res["query"]["resizes"]
    dg.release()


def test_host_target_down_to_one_and_back(rt, coop_mod, gg):
    """The target drops to one workgroup (workgroup 0 alone, the master at
    every barrier, must still see the host's target) and comes back: the
    joiners are admitted and the launch ends at (nearly) full size with the
    oracle's levels."""
    import time
    import torch
    c = coop_mod
    g = gg.rmat(18, 16, seed=3)
    dg = rt.graph(g)
    roots = np.resize(gg.sources(g, 3, 16), 2000).astype(np.uint32)
    d_roots = rt._roots(roots)
    lv = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    say(f"bfs rmat18 x{len(roots)}: target 1, then back to N")
    h = c.coop_bfs(rt.rt, dg.handle, d_roots, len(roots), lv, g.n, o)
    n = c.coop_handle_groups(h)
    time.sleep(0.01)
    c.coop_set_target(h, 1)
    time.sleep(0.02)
    c.coop_set_target(h, n)
    c.coop_fork_groups(h, n)
    rc, st = c.coop_wait(h)
    say(f"  kernel {st['kernel_ms']:.1f} ms kills={st['kills']} forks={st['forks']} "
        f"min={st['min_groups']} final={st['final_groups']}")
    assert rc == 0, c.coop_strerror(rc)
    check_rows(lv, roots, g)
    # the hardware deals joiners over the shader engines, so one may wait for
    # a unit on its own engine while another engine has one idle: nearly N
    assert st["min_groups"] == 1 and st["final_groups"] >= n - 8
    dg.release()


@pytest.mark.parametrize("window", [0, 300])
def test_admission_ring_flood(rt, coop_mod, gg, window):
    """Far more joiner workgroups than the admission ring holds (12000
    against 8192 entries) take slots and give up while the target leaves no
    room, the state surplus joiners reach under co-tasks. A joiner whose
    slot lies beyond the ring's window leaves without touching it, the
    master admits only joiners still waiting, and the levels match the
    oracle. window=300 (just above N) makes a full ring the common case; 0
    is the default window (8192 - N)."""
    import time
    import torch
    c = coop_mod
    g = gg.rmat(18, 16, seed=3)
    dg = rt.graph(g)
    roots = np.resize(gg.sources(g, 3, 16), 2000).astype(np.uint32)
    d_roots = rt._roots(roots)
    lv = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
    cus = rt.info["compute_units"]
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE, join_window=window)
    say(f"bfs rmat18 x{len(roots)}: 12000 joiners at half target, join_window={window}")
    h = c.coop_bfs(rt.rt, dg.handle, d_roots, len(roots), lv, g.n, o)
    time.sleep(0.01)
    c.coop_set_target(h, cus // 2)
    time.sleep(0.01)
    c.coop_fork_groups(h, 12000)
    time.sleep(0.06)
    c.coop_set_target(h, cus)
    c.coop_fork_groups(h, cus // 2)
    rc, st = c.coop_wait(h)
    say(f"  kernel {st['kernel_ms']:.1f} ms kills={st['kills']} forks={st['forks']} "
        f"join_full={st['join_full']} min_groups={st['min_groups']}")
    assert rc == 0, c.coop_strerror(rc)
    check_rows(lv, roots, g)
    assert st["kills"] > 0 and st["min_groups"] <= cus // 2
    if window:
        assert st["join_full"] > 0
    dg.release()
