"""GPU parity at the benchmark's full sizes and launch configuration, every
output against the oracle element by element:

* BFS on R-MAT scale 22 (edge factor 16, seed 3; n = 4,194,304), the
  benchmark's first timed launch: eight seeded sources in one persistent
  launch of all resident 1024-thread workgroups, cooperative with the
  host-driven scheduler and plain;
* the same graph while co-tasks take half the compute units every 2 ms
  (kills and joiner grids during the traversal);
* frontier Bellman-Ford SSSP on the 1024 x 1024 grid (weights U[1,1000],
  seed 2) from vertex 0, cooperative with the host-driven scheduler and
  plain, and under the benchmark's seeded random kill/fork schedule
  (killed workgroups queue again as joiners)."""
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


@pytest.fixture(scope="module")
def rmat22(rt, gg):
    say("generating R-MAT scale 22 (seed 3)")
    g = gg.rmat(22, 16, seed=3)
    dg = rt.graph(g)
    roots = [int(r) for r in gg.sources(g, 3, 16)[8:16]]     # the first timed launch
    say(f"  n={g.n} arcs={g.arcs}; oracle BFS for roots {roots}")
    exp = {r: oracle.bfs(g, r) for r in roots}
    yield g, dg, roots, exp
    dg.release()


# "slot_sums": the level counts summed from the statistics slots instead of
# coming with the barrier arrivals (the default at this size)
@pytest.mark.parametrize("mode", ["coop_host", "plain", "coop_host_slot_sums"])
def test_bfs_rmat22_bench_launch(rt, coop_mod, rmat22, mode):
    c = coop_mod
    g, dg, roots, exp = rmat22
    o = {"coop_host": lambda: c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE),
         "plain": lambda: c.make_opts(c.COOP_MODE_PLAIN),
         "coop_host_slot_sums": lambda: c.make_opts(c.COOP_MODE_COOP,
                                                    flags=c.COOP_F_HOST_SCHEDULE | c.COOP_F_SLOT_SUMS)}[mode]()
    say(f"bfs rmat22 {mode}: 8 sources in one launch")
    rc, out, st = rt.bfs(dg, roots, o)
    assert rc == 0, c.coop_strerror(rc)
    assert st["grid"] == rt.info["compute_units"]
    got = out.cpu().numpy().view(np.uint32)
    for i, r in enumerate(roots):
        assert np.array_equal(got[i], exp[r]), f"root {r}"
    say(f"  kernel {st['kernel_ms']:.3f} ms, {st['levels']} levels")


def test_bfs_rmat22_with_cotasks(rt, coop_mod, rmat22):
    """48 traversals (the eight sources six times) in one cooperative launch
    while the injector takes half the compute units for 0.5 ms every 2 ms."""
    import torch
    c = coop_mod
    g, dg, roots, exp = rmat22
    seq = roots * 6
    d_roots = rt._roots(np.array(seq, dtype=np.uint32))
    out = torch.empty(len(seq) * g.n, dtype=torch.int32, device="cuda")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    cus = rt.info["compute_units"]
    say(f"bfs rmat22 x{len(seq)} with co-tasks")
    h = c.coop_bfs(rt.rt, dg.handle, d_roots, len(seq), out, g.n, o)
    c.coop_injector_start(rt.rt, h, groups=cus // 2, busy_ns=500_000, period_ns=2_000_000)
    rc, st = c.coop_wait(h)
    irc, cst = c.coop_injector_stop(rt.rt)
    assert rc == 0 and irc == 0, (c.coop_strerror(rc), c.coop_strerror(irc))
    say(f"  kernel {st['kernel_ms']:.1f} ms kills={st['kills']} forks={st['forks']} co-tasks={cst['count']} "
        f"p99={cst['latency_p99_ms']:.3f} ms")
    got = out.cpu().numpy().view(np.uint32).reshape(len(seq), g.n)
    for i, r in enumerate(seq):
        assert np.array_equal(got[i], exp[r]), f"traversal {i} root {r}"
    assert cst["count"] >= 3 and st["kills"] > 0


@pytest.fixture(scope="module")
def grid1024(rt, gg):
    g = gg.add_weights(gg.grid(1024, 1024), 2, 1, 1000)
    dg = rt.graph(g)
    exp = oracle.sssp(g, 0)
    yield g, dg, exp
    dg.release()


@pytest.mark.parametrize("mode", ["coop_host", "plain", "random"])
def test_sssp_grid1024_bench_launch(rt, coop_mod, grid1024, mode):
    c = coop_mod
    g, dg, exp = grid1024
    o = {"coop_host": lambda: c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE),
         "plain": lambda: c.make_opts(c.COOP_MODE_PLAIN),
         "random": lambda: c.make_opts(c.COOP_MODE_COOP,
                                       flags=c.COOP_F_RANDOM_SCHEDULE | c.COOP_F_PARK_KILLED,
                                       sched_seed=1, sched_p=0.25)}[mode]()
    say(f"sssp grid1024 {mode}")
    rc, d, st = rt.sssp(dg, [0], o)
    assert rc == 0, c.coop_strerror(rc)
    assert np.array_equal(d.cpu().numpy(), exp)
    say(f"  kernel {st['kernel_ms']:.1f} ms, {st['levels']} rounds, kills={st['kills']}")
    if mode == "random":
        assert st["kills"] > 0
