"""GPU parity of the work-stealing octree (the paper's work-stealing class):
the points in final order and the leaves must equal the oracle's exactly,
in plain and cooperative launches, while the scheduler target moves and
joiner grids arrive, and while co-tasks take compute units."""
import sys
import threading
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
    yield r
    r.close()


@pytest.fixture(scope="module")
def coop_mod():
    from paper_1707_01989_amd import coop
    return coop


def check(rt, x, y, z, cap, opts, what):
    say(f"octree {what}: n={len(x)} cap={cap}")
    rc, pts, lv, st = rt.octree(x, y, z, cap, opts)
    assert rc == 0, f"{what}: error {rc}"
    exp_pts, exp_lv = oracle.octree(x, y, z, cap)
    assert np.array_equal(pts, exp_pts), f"{what}: point order differs"
    assert np.array_equal(lv, exp_lv), f"{what}: leaves differ"
    say(f"  {st['kernel_ms']:.2f} ms, {st['levels']} splits, {st['rows']} leaves, {st['arcs']} steals, "
        f"groups [{st['min_groups']},{st['max_groups']}]")
    return st


@pytest.mark.parametrize("kind,n,cap,seed", [("uniform", 20000, 8, 1), ("clustered", 100000, 16, 2),
                                             ("uniform", 1000000, 32, 3), ("clustered", 500000, 4, 4)])
@pytest.mark.parametrize("mode", ["plain", "coop"])
def test_octree_parity(rt, coop_mod, gg, kind, n, cap, seed, mode):
    c = coop_mod
    x, y, z = gg.points(n, seed, kind)
    o = c.make_opts(c.COOP_MODE_PLAIN if mode == "plain" else c.COOP_MODE_COOP)
    st = check(rt, x, y, z, cap, o, f"{kind} {mode}")
    assert st["levels"] > 0 and st["rows"] > 0


def test_octree_edge_cases(rt, coop_mod):
    c = coop_mod
    o = c.make_opts(c.COOP_MODE_COOP)
    small = np.array([7, 3, 9], dtype=np.uint32)
    check(rt, small, small, small, 3, o, "root is a leaf")
    same = np.full(5000, 777777, dtype=np.uint32)
    check(rt, same, same, same, 16, o, "identical points (leaf at depth 21)")
    e = np.zeros(0, dtype=np.uint32)
    rc, pts, lv, st = rt.octree(e, e, e, 4, o)
    assert rc == 0 and pts.shape == (0, 4) and lv.shape[0] == 0


def test_octree_under_moving_target(rt, coop_mod, gg):
    """Workgroups leave (kill in any order, by shader engine) and joiner
    grids take free slots while the build runs."""
    c = coop_mod
    x, y, z = gg.points(4000000, 9, "clustered")
    exp_pts, exp_lv = oracle.octree(x, y, z, 8)
    import torch
    n = len(x)
    dx, dy, dz = (torch.from_numpy(v.view(np.int32)).cuda() for v in (x, y, z))
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    leaves = torch.empty((n, 8), dtype=torch.int32, device="cuda")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    say("octree clustered 4M under a moving target")
    h = c.coop_octree(rt.rt, dx, dy, dz, n, 8, out, leaves, n, o)
    N = c.coop_handle_groups(h)
    stop = threading.Event()

    def scheduler():
        k = 0
        while not stop.is_set():
            c.coop_set_target(h, max(1, N // 4) if k % 2 == 0 else N)
            if k % 2 == 1:
                c.coop_fork_groups(h, N // 2)
            k += 1
            time.sleep(0.002)

    th = threading.Thread(target=scheduler)
    th.start()
    try:
        rc, st = c.coop_wait(h)
    finally:
        stop.set()
        th.join()
    assert rc == 0, c.coop_strerror(rc)
    say(f"  {st['kernel_ms']:.1f} ms kills={st['kills']} forks={st['forks']} groups [{st['min_groups']},"
        f"{st['max_groups']}] steals={st['arcs']}")
    pts = out.cpu().numpy().view(np.uint32)
    lv = leaves.cpu().numpy().view(np.uint32)[: st["rows"], :5]
    lv = lv[np.argsort(lv[:, 0], kind="stable")]
    assert np.array_equal(pts, exp_pts) and np.array_equal(lv, exp_lv)
    assert st["kills"] > 0


def test_octree_with_cotasks(rt, coop_mod, gg):
    c = coop_mod
    x, y, z = gg.points(4000000, 10, "uniform")
    exp_pts, exp_lv = oracle.octree(x, y, z, 4)
    import torch
    n = len(x)
    dx, dy, dz = (torch.from_numpy(v.view(np.int32)).cuda() for v in (x, y, z))
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    leaves = torch.empty((n, 8), dtype=torch.int32, device="cuda")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    cus = rt.info["compute_units"]
    say("octree uniform 4M with co-tasks")
    h = c.coop_octree(rt.rt, dx, dy, dz, n, 4, out, leaves, n, o)
    c.coop_injector_start(rt.rt, h, groups=cus // 2, busy_ns=200_000, period_ns=1_000_000)
    rc, st = c.coop_wait(h)
    irc, cst = c.coop_injector_stop(rt.rt)
    assert rc == 0 and irc == 0, (c.coop_strerror(rc), c.coop_strerror(irc))
    say(f"  {st['kernel_ms']:.1f} ms co-tasks={cst['count']} latency p50={cst['latency_p50_ms']:.3f} "
        f"p99={cst['latency_p99_ms']:.3f} ms kills={st['kills']}")
    pts = out.cpu().numpy().view(np.uint32)
    lv = leaves.cpu().numpy().view(np.uint32)[: st["rows"], :5]
    lv = lv[np.argsort(lv[:, 0], kind="stable")]
    assert np.array_equal(pts, exp_pts) and np.array_equal(lv, exp_lv)
