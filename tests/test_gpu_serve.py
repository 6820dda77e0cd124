"""GPU parity of the query server: BFS and SSSP queries admitted into one
persistent launch as slots free up. Every query's result must equal the
oracle's and be the same whether the query ran alone or in a mix with
others, under any team sizing, slot budget and kill/fork schedule."""
import sys
import time

import numpy as np
import pytest

import oracle
from tests.conftest import gpu_available

# every wait below is bounded well inside the test's own time limit, so a
# stuck query fails the test and coop_server_destroy still stops the launch
pytestmark = [
    pytest.mark.gpu,
    pytest.mark.timeout(400),
    pytest.mark.skip(reason="two GPU runs of these tests ended the box with a GPU memory fault or hung queue "
                            "(the second after a host copy that could not find a free CU was ruled out); the "
                            "cause is not shown yet, so the server stays off the GPU (coop_server_create "
                            "refuses to start) until it is"),
]


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


@pytest.fixture(scope="module")
def graphs(rt, gg):
    gs = [gg.add_weights(gg.er(20000, 12, 41), 5, 1, 1000),
          gg.add_weights(gg.grid(96, 128), 6, 1, 1000),
          gg.add_weights(gg.rmat(14, 8, seed=7), 7, 1, 255),
          gg.add_weights(gg.disjoint_union(gg.er(3000, 6, 3), gg.path(500)), 8, 1, 50)]
    dgs = [rt.graph(g) for g in gs]
    yield gs, dgs
    for d in dgs:
        d.release()


def make_queries(gs, count, seed):
    rng = np.random.default_rng(seed)
    qs = []
    for _ in range(count):
        gi = int(rng.integers(len(gs)))
        kind = int(rng.integers(1, 3))
        deg = gs[gi].degrees()
        cand = np.nonzero(deg > 0)[0]
        qs.append((gi, kind, int(cand[rng.integers(len(cand))])))
    return qs


def expected(gs, q, cache):
    if q not in cache:
        gi, kind, src = q
        cache[q] = oracle.bfs(gs[gi], src) if kind == 1 else oracle.sssp(gs[gi], src).view(np.uint32)
    return cache[q]


def run_queries(c, srv, dgs, qs, spacing_s=0.0):
    import torch
    outs, tickets = [], []
    for gi, kind, src in qs:
        out = torch.empty(dgs[gi].n, dtype=torch.int32, device="cuda")
        tickets.append(c.coop_server_submit(srv, dgs[gi].handle, kind, src, out))
        outs.append(out)
        if spacing_s:
            time.sleep(spacing_s)
    lats = []
    for t in tickets:
        rc, lat = c.coop_server_wait(srv, t, 20000.0)
        assert rc == 0, c.coop_strerror(rc)
        lats.append(lat)
    return [o.cpu().numpy().view(np.uint32) for o in outs], lats


@pytest.mark.parametrize("cfg", ["default", "big_teams", "one_slot", "plain"])
def test_serve_alone_vs_mix(rt, coop_mod, graphs, cfg):
    c = coop_mod
    gs, dgs = graphs
    kw = {"default": {}, "big_teams": {"team_arcs_bfs": 1 << 13, "team_arcs_sssp": 1 << 15, "team_max": 8},
          "one_slot": {"max_queries": 1, "team_arcs_bfs": 1 << 14},
          "plain": {"mode": c.COOP_MODE_PLAIN, "team_arcs_bfs": 1 << 15}}[cfg]
    qs = make_queries(gs, 40, 3)
    cache = {}
    srv = c.coop_server_create(rt.rt, [d.handle for d in dgs], 1 << 30, c.make_server_cfg(**kw))
    try:
        say(f"serve alone vs mix cfg={cfg}: {c.coop_server_stats(srv)['slots']} slots")
        alone = [run_queries(c, srv, dgs, [q])[0][0] for q in qs]
        mix, lats = run_queries(c, srv, dgs, qs)
        for i, q in enumerate(qs):
            exp = expected(gs, q, cache)
            assert np.array_equal(alone[i], exp), f"alone query {i} {q}"
            assert np.array_equal(mix[i], exp), f"mixed query {i} {q}"
        st = c.coop_server_stats(srv)
        say(f"  completed={st['completed']} p50={st['latency_p50_ms']} p99={st['latency_p99_ms']} "
            f"wait p99={st['wait_p99_ms']:.3f}")
        assert st["completed"] == 2 * len(qs) and st["error"] == 0
    finally:
        assert c.coop_server_destroy(srv) == 0


def test_serve_poisson_with_target_changes(rt, coop_mod, graphs):
    """Queries arrive while the scheduler target moves (workgroups leave
    between queries and at team barriers) and joiner grids come back."""
    c = coop_mod
    gs, dgs = graphs
    qs = make_queries(gs, 60, 11)
    cache = {}
    cfg = c.make_server_cfg(flags=c.COOP_F_HOST_SCHEDULE, team_arcs_bfs=1 << 13, team_arcs_sssp=1 << 14,
                            team_max=16, max_queries=6)
    srv = c.coop_server_create(rt.rt, [d.handle for d in dgs], 1 << 30, cfg)
    try:
        h = c.coop_server_handle(srv)
        n = c.coop_handle_groups(h)
        import threading
        stop = threading.Event()

        def scheduler():
            k = 0
            while not stop.is_set():
                c.coop_set_target(h, max(1, n // 4) if k % 2 == 0 else n)
                if k % 2 == 1:
                    c.coop_fork_groups(h, n // 2)
                k += 1
                time.sleep(0.003)
            c.coop_set_target(h, n)
            c.coop_fork_groups(h, n)

        th = threading.Thread(target=scheduler)
        th.start()
        try:
            rng = np.random.default_rng(5)
            import torch
            outs, tickets = [], []
            for gi, kind, src in qs:
                out = torch.empty(dgs[gi].n, dtype=torch.int32, device="cuda")
                tickets.append(c.coop_server_submit(srv, dgs[gi].handle, kind, src, out))
                outs.append(out)
                time.sleep(float(rng.exponential(0.0005)))
            for t in tickets:
                rc, _ = c.coop_server_wait(srv, t, 20000.0)
                assert rc == 0, c.coop_strerror(rc)
        finally:
            stop.set()
            th.join()
        for i, q in enumerate(qs):
            assert np.array_equal(outs[i].cpu().numpy().view(np.uint32), expected(gs, q, cache)), f"query {i} {q}"
        st = c.coop_server_stats(srv)
        say(f"  kills={st['kills']} forks={st['forks']} min={st['min_groups']} max={st['max_groups']}")
        assert st["kills"] > 0
        assert st["min_groups"] >= 16
    finally:
        assert c.coop_server_destroy(srv) == 0


def test_serve_with_cotask_injector(rt, coop_mod, graphs):
    c = coop_mod
    gs, dgs = graphs
    qs = make_queries(gs, 80, 21)
    cache = {}
    cfg = c.make_server_cfg(flags=c.COOP_F_HOST_SCHEDULE, team_arcs_bfs=1 << 14)
    srv = c.coop_server_create(rt.rt, [d.handle for d in dgs], 1 << 30, cfg)
    try:
        h = c.coop_server_handle(srv)
        cus = rt.info["compute_units"]
        c.coop_injector_start(rt.rt, h, groups=cus // 2, busy_ns=200_000, period_ns=2_000_000)
        try:
            outs, lats = run_queries(c, srv, dgs, qs, spacing_s=0.0005)
        finally:
            irc, cst = c.coop_injector_stop(rt.rt)
        assert irc == 0, c.coop_strerror(irc)
        say(f"  co-tasks={cst['count']} latency p50={cst['latency_p50_ms']:.3f} p99={cst['latency_p99_ms']:.3f} ms")
        assert cst["count"] > 0
        for i, q in enumerate(qs):
            assert np.array_equal(outs[i], expected(gs, q, cache)), f"query {i} {q}"
    finally:
        assert c.coop_server_destroy(srv) == 0


def test_serve_rejects_bad_queries(rt, coop_mod, graphs, gg):
    import torch
    c = coop_mod
    gs, dgs = graphs
    unweighted = rt.graph(gg.er(100, 4, 1))
    srv = c.coop_server_create(rt.rt, [dgs[0].handle, unweighted.handle], 1 << 28)
    try:
        out = torch.empty(dgs[0].n, dtype=torch.int32, device="cuda")
        with pytest.raises(c.CoopError):
            c.coop_server_submit(srv, dgs[1].handle, c.COOP_QUERY_BFS, 0, out)      # not served
        with pytest.raises(c.CoopError):
            c.coop_server_submit(srv, dgs[0].handle, c.COOP_QUERY_BFS, dgs[0].n, out)
        with pytest.raises(c.CoopError):
            c.coop_server_submit(srv, unweighted.handle, c.COOP_QUERY_SSSP, 0, out)
        with pytest.raises(c.CoopError):
            c.coop_server_submit(srv, dgs[0].handle, 9, 0, out)
        t = c.coop_server_submit(srv, unweighted.handle, c.COOP_QUERY_BFS, 3, out)
        rc, _ = c.coop_server_wait(srv, t, 20000.0)
        assert rc == 0
        assert np.array_equal(out.cpu().numpy().view(np.uint32)[:100], oracle.bfs(gg.er(100, 4, 1), 3))
    finally:
        assert c.coop_server_destroy(srv) == 0
        unweighted.release()
    with pytest.raises(c.CoopError):           # a budget that holds no slot
        c.coop_server_create(rt.rt, [dgs[0].handle], 1024)
