"""GPU test of coop_bfs_noalloc, the BFS entry point that allocates nothing
(its scratch is one static device array per GPU): called through the C
ABI, its levels must equal coop_bfs's on the same inputs, element by
element, on two calls in a row, the second with a smaller graph, so the
second call runs over what the first left in the array."""
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


def noalloc_levels(c, rt, dg, roots, opts, stride=True):
    """Levels of every source from coop_bfs_noalloc (one row per source)
    and the status word the launch wrote."""
    import torch
    d_roots = rt._roots(roots)
    k = d_roots.numel()
    out = torch.full((k * dg.n,), 7, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    c.coop_bfs_noalloc(rt.rt, dg.handle, d_roots, k, out, dg.n if (stride and k > 1) else 0, opts, status,
                       stream)
    torch.cuda.synchronize()
    return int(status.item()), out.cpu().numpy().view(np.uint32).reshape(k, dg.n)


def alloc_levels(c, rt, dg, roots, opts):
    rc, out, _ = rt.bfs(dg, roots, opts)
    assert rc == 0, c.coop_strerror(rc)
    return out.cpu().numpy().view(np.uint32).reshape(len(roots), dg.n)


@pytest.mark.parametrize("mode", ["plain", "coop", "coop_random"])
def test_noalloc_matches_coop_bfs_twice(rt, coop_mod, gg, mode):
    c = coop_mod
    opts = {"plain": c.make_opts(c.COOP_MODE_PLAIN),
            "coop": c.make_opts(c.COOP_MODE_COOP),
            "coop_random": c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_RANDOM_SCHEDULE | c.COOP_F_PARK_KILLED,
                                       sched_seed=5, sched_p=0.3)}[mode]
    big = gg.rmat(16, 16, seed=9)                     # several heavy strips, bottom-up levels
    small = gg.disjoint_union(gg.er(3000, 6, 3), gg.path(700))
    for name, g, roots in (("rmat16", big, gg.sources(big, 4, 3)), ("er3000+path", small, [0, 3100, 2999])):
        say(f"noalloc mode={mode} graph={name} n={g.n} roots={list(map(int, roots))}")
        dg = rt.graph(g)
        try:
            st, got = noalloc_levels(c, rt, dg, roots, opts)
            assert st == 0, c.coop_strerror(st)
            exp = alloc_levels(c, rt, dg, roots, opts)
            assert np.array_equal(got, exp), f"{name}: differs from coop_bfs"
            assert np.array_equal(got[0], oracle.bfs(g, int(roots[0]))), f"{name}: differs from the oracle"
        finally:
            dg.release()


def test_noalloc_refusals_and_status(rt, coop_mod, gg):
    import torch
    c = coop_mod
    g = gg.er(200000, 16, 7)
    dg = rt.graph(g)
    try:
        roots = rt._roots([0])
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        # a host-driven target needs pinned memory: refused
        with pytest.raises(c.CoopError) as e:
            c.coop_bfs_noalloc(rt.rt, dg.handle, roots, 1, out, 0,
                               c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE), status)
        assert e.value.code == c.COOP_E_INVALID
        # one-arc strips of every vertex need 16 B per arc, more than the array holds
        with pytest.raises(c.CoopError) as e:
            c.coop_bfs_noalloc(rt.rt, dg.handle, roots, 1, out, 0,
                               c.make_opts(c.COOP_MODE_COOP, heavy_threshold=1, strip=1), status)
        assert e.value.code == c.COOP_E_TOO_BIG
        # a source outside the graph: the launch reports it in the status word
        bad = rt._roots([g.n + 5])
        c.coop_bfs_noalloc(rt.rt, dg.handle, bad, 1, out, 0, c.make_opts(c.COOP_MODE_COOP), status)
        torch.cuda.synchronize()
        assert int(status.item()) == c.COOP_E_INVALID
        # and the next call on the same array is clean again
        st, got = noalloc_levels(c, rt, dg, [0], c.make_opts(c.COOP_MODE_COOP))
        assert st == 0 and np.array_equal(got[0], oracle.bfs(g, 0))
    finally:
        dg.release()
