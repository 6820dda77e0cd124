"""GPU parity of the batched launch: many graph instances in one persistent
launch, each run by a team of workgroups with its own barrier. Every
instance's BFS levels, colours and MIS flags must equal the oracle's, for
any team sizing, group size, BFS direction rule and kill/fork schedule."""
import sys

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
    yield r
    r.close()


@pytest.fixture(scope="module")
def coop_mod():
    from paper_1707_01989_amd import coop
    return coop


def small_mix(gg):
    """Uneven instances: ER of several sizes and degrees, grids, a tree, a
    path, a star, a complete graph, graphs with isolated vertices."""
    gs = []
    for i in range(24):
        n = [64, 300, 1000, 2500, 7000, 20000][i % 6]
        gs.append(gg.er(n, 4 + (i * 7) % 29, 500 + i))
    gs += [gg.grid(40, 60), gg.binary_tree(1023), gg.path(777), gg.star(500), gg.complete(90),
           gg.disjoint_union(gg.empty(5), gg.er(400, 6, 9)), gg.empty(33), gg.rmat(12, 8, seed=5)]
    return gs


def check(gs, outs, roots, seeds, ops, coop):
    for i, g in enumerate(gs):
        if ops & coop.COOP_BATCH_BFS:
            got = outs[i]["level"].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, oracle.bfs(g, int(roots[i]))), f"bfs instance {i} ({g.name})"
        if ops & coop.COOP_BATCH_COLOR:
            got = outs[i]["colour"].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, oracle.color(g, int(seeds[i]))), f"colour instance {i} ({g.name})"
        if ops & coop.COOP_BATCH_MIS:
            got = outs[i]["in_set"].cpu().numpy()
            assert np.array_equal(got, oracle.mis(g, int(seeds[i]))), f"mis instance {i} ({g.name})"


TUNES = {
    "default": {},
    "teams_of_many": {"team_arcs": 1 << 10, "team_max": 16},
    "small_groups": {"group_size": 256, "team_arcs": 1 << 12},
    "top_down": {"direction_opt": 0, "team_arcs": 1 << 13},
    "one_group_each": {"team_arcs": 1 << 40},
    "few_groups": {"num_groups": 6, "team_max": 3, "team_arcs": 1 << 12},
}


@pytest.mark.parametrize("tune", list(TUNES))
@pytest.mark.parametrize("ops", ["bfs_color", "bfs_mis"])
def test_batch_small_mix(rt, coop_mod, gg, tune, ops):
    c = coop_mod
    gs = small_mix(gg)
    op = c.COOP_BATCH_BFS | (c.COOP_BATCH_COLOR if ops == "bfs_color" else c.COOP_BATCH_MIS)
    roots = [(7 * i) % g.n for i, g in enumerate(gs)]
    seeds = [1000 + 3 * i for i in range(len(gs))]
    dgs = [rt.graph(g) for g in gs]
    items, outs = rt.batch_items(dgs, op, roots, seeds)
    say(f"batch small mix tune={tune} ops={ops} instances={len(gs)}")
    for mode in ("plain", "coop"):
        rc, st = rt.batch(items, c.make_tune(**TUNES[tune]), c.make_opts(getattr(c, f"COOP_MODE_{mode.upper()}")))
        assert rc == 0, c.coop_strerror(rc)
        check(gs, outs, roots, seeds, op, c)
        say(f"  {mode}: {st['kernel_ms']:.3f} ms barriers={st['barriers']} levels={st['levels']}")
    for dg in dgs:
        dg.release()


@pytest.mark.parametrize("seed", range(3))
def test_batch_random_kills_and_joiners(rt, coop_mod, gg, seed):
    """Workgroups leave between instances under a seeded random schedule
    (never below the largest team) and a joiner grid brings new ones in;
    results do not change."""
    import torch
    c = coop_mod
    gs = small_mix(gg) + [gg.er(30000 + 1000 * k, 12, 70 + k) for k in range(8)]
    op = c.COOP_BATCH_BFS | c.COOP_BATCH_COLOR
    roots = [0] * len(gs)
    seeds = list(range(len(gs)))
    dgs = [rt.graph(g) for g in gs]
    items, outs = rt.batch_items(dgs, op, roots, seeds)
    say(f"batch random kills seed={seed}")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_RANDOM_SCHEDULE, sched_seed=seed, sched_p=0.5)
    t = c.make_tune(team_arcs=1 << 13, team_max=4, num_groups=40, group_size=256)
    h = c.coop_batch_run(rt.rt, items, t, o)
    c.coop_fork_groups(h, 24)
    rc, st = c.coop_wait(h)
    assert rc == 0, c.coop_strerror(rc)
    torch.cuda.synchronize()
    check(gs, outs, roots, seeds, op, c)
    say(f"  kills={st['kills']} forks={st['forks']} min={st['min_groups']} max={st['max_groups']}")
    assert st["kills"] > 0
    assert st["min_groups"] >= 4
    for dg in dgs:
        dg.release()


def test_batch_host_target(rt, coop_mod, gg):
    """The host target shrinks the batch between instances; restoring it and
    forking brings workgroups back."""
    import time
    c = coop_mod
    gs = [gg.er(20000 + 500 * k, 16, 300 + k) for k in range(64)]
    op = c.COOP_BATCH_BFS | c.COOP_BATCH_COLOR
    dgs = [rt.graph(g) for g in gs]
    roots = [0] * len(gs)
    seeds = list(range(len(gs)))
    items, outs = rt.batch_items(dgs, op, roots, seeds)
    say("batch host target")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    t = c.make_tune(team_arcs=1 << 40, num_groups=16, team_max=2, group_size=256)
    h = c.coop_batch_run(rt.rt, items, t, o)
    c.coop_set_target(h, 4)
    time.sleep(0.002)
    c.coop_set_target(h, 16)
    c.coop_fork_groups(h, 8)
    rc, st = c.coop_wait(h)
    assert rc == 0, c.coop_strerror(rc)
    check(gs, outs, roots, seeds, op, c)
    say(f"  kills={st['kills']} forks={st['forks']} min={st['min_groups']}")
    for dg in dgs:
        dg.release()


def test_batch_rejects_bad_items(rt, coop_mod, gg):
    c = coop_mod
    g = gg.er(100, 4, 1)
    dg = rt.graph(g)
    items, _ = rt.batch_items([dg], c.COOP_BATCH_BFS)
    bad = c.coop_batch_item(graph=dg.handle, ops=c.COOP_BATCH_BFS, bfs_root=100, d_level=items[0].d_level)
    with pytest.raises(c.CoopError):
        c.coop_batch_run(rt.rt, [bad])
    both = c.coop_batch_item(graph=dg.handle, ops=c.COOP_BATCH_COLOR | c.COOP_BATCH_MIS,
                             d_colour=items[0].d_level, d_in_set=items[0].d_level)
    with pytest.raises(c.CoopError):
        c.coop_batch_run(rt.rt, [both])
    with pytest.raises(c.CoopError):          # team cap above the launch size
        c.coop_batch_run(rt.rt, items, c.make_tune(num_groups=4, team_max=8))
    dg.release()


def test_batch_autotune(rt, coop_mod, gg):
    c = coop_mod
    gs = [gg.er(n, d, 900 + i) for i, (n, d) in enumerate([(2000, 8), (50000, 16), (120000, 24), (9000, 30)] * 6)]
    dgs = [rt.graph(g) for g in gs]
    op = c.COOP_BATCH_BFS | c.COOP_BATCH_COLOR
    items, outs = rt.batch_items(dgs, op)
    say("batch autotune")
    best, best_ms, def_ms = c.coop_batch_autotune(rt.rt, items, stride=2, reps=3)
    say(f"  best={best.as_dict()} {best_ms:.3f} ms (default {def_ms:.3f} ms)")
    assert best_ms <= def_ms * 1.02
    again, ms2, d2 = c.coop_batch_autotune(rt.rt, items, stride=2, reps=3)
    assert again.as_dict() == best.as_dict() and d2 < 0        # served from the cache
    # the cache survives a save, a clear and a load (a later process)
    import tempfile, os
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    assert c.coop_tune_cache_save(path) >= 1
    c.coop_tune_cache_clear()
    assert c.coop_tune_cache_load(path) >= 1
    third, _, d3 = c.coop_batch_autotune(rt.rt, items, stride=2, reps=3)
    assert third.as_dict() == best.as_dict() and d3 < 0
    rc, st = rt.batch(items, best)
    assert rc == 0
    check(gs, outs, [0] * len(gs), list(range(len(gs))), op, c)
    for dg in dgs:
        dg.release()


def test_batch_full_er512(rt, coop_mod, gg):
    """The full batched workload: 512 ER instances, n log-uniform in
    [2^10, 2^18), average degree U[4, 32], seeds 1000 + i; BFS from vertex 0,
    then greedy colouring with priority seed i, in one launch; every
    instance checked against the oracle."""
    c = coop_mod
    gs = gg.er_batch(512, 1000, workers=16)
    say(f"batch er512: n={sum(g.n for g in gs)} arcs={sum(g.arcs for g in gs)}")
    dgs = [rt.graph(g) for g in gs]
    op = c.COOP_BATCH_BFS | c.COOP_BATCH_COLOR
    items, outs = rt.batch_items(dgs, op)
    for mode in ("plain", "coop"):
        rc, st = rt.batch(items, None, c.make_opts(getattr(c, f"COOP_MODE_{mode.upper()}")))
        assert rc == 0, c.coop_strerror(rc)
        say(f"  {mode}: {st['kernel_ms']:.3f} ms barriers={st['barriers']}")
    check(gs, outs, [0] * len(gs), list(range(len(gs))), op, c)
    for dg in dgs:
        dg.release()
