"""Several cooperative launches at once: a host sharer gives each its
weighted share of the resident workgroups (as scheduler targets) and forks
joiners when a share grows. Every output must equal the oracle's, however
the launches were resized."""
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


@pytest.mark.parametrize("weights", [(1, 1), (3, 1)])
def test_bfs_and_sssp_share_the_gpu(rt, coop_mod, gg, weights):
    import torch
    c = coop_mod
    ga = gg.rmat(18, 16, seed=3)
    gb = gg.add_weights(gg.grid(256, 256), 2, 1, 1000)
    da, db = rt.graph(ga), rt.graph(gb)
    roots = np.resize(gg.sources(ga, 3, 16), 400).astype(np.uint32)
    d_roots = rt._roots(roots)
    d_src = rt._roots(np.array([0], dtype=np.uint32))
    lv = torch.empty(ga.n, dtype=torch.int32, device="cuda")
    dist = torch.empty(gb.n, dtype=torch.int32, device="cuda")
    o = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    sb = torch.cuda.Stream()
    say(f"share: bfs rmat18 x{len(roots)} (weight {weights[0]}) + sssp grid256 (weight {weights[1]})")
    c.coop_share_start(rt.rt, 100)
    try:
        ha = c.coop_bfs(rt.rt, da.handle, d_roots, len(roots), lv, 0, o)
        c.coop_share_add(rt.rt, ha, weights[0])
        hb = c.coop_sssp(rt.rt, db.handle, d_src, 1, dist, 0, o, sb)
        c.coop_share_add(rt.rt, hb, weights[1])
        rcb, stb = c.coop_wait(hb)
        rca, sta = c.coop_wait(ha)
    finally:
        rcs, sst = c.coop_share_stop(rt.rt)
    assert rca == 0 and rcb == 0 and rcs == 0, (c.coop_strerror(rca), c.coop_strerror(rcb), c.coop_strerror(rcs))
    say(f"  bfs {sta['kernel_ms']:.1f} ms M in [{sta['min_groups']},{sta['max_groups']}] kills={sta['kills']} "
        f"forks={sta['forks']}; sssp {stb['kernel_ms']:.1f} ms M in [{stb['min_groups']},{stb['max_groups']}]; {sst}")
    assert np.array_equal(lv.cpu().numpy().view(np.uint32), oracle.bfs(ga, int(roots[-1])))
    assert np.array_equal(dist.cpu().numpy(), oracle.sssp(gb, 0))
    n = rt.info["compute_units"]
    # the traversal gave workgroups up while the other launch ran, and got
    # some back (joiners) after it ended
    assert sta["kills"] > 0 and sta["min_groups"] < n
    assert stb["max_groups"] <= n
    assert sst["launches"] == 2 and sst["target_updates"] >= 2
    da.release()
    db.release()


def test_share_rejects_bad_use(rt, coop_mod, gg):
    c = coop_mod
    g = gg.er(1000, 4, 1)
    dg = rt.graph(g)
    import torch
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    plain = c.make_opts(c.COOP_MODE_PLAIN)
    h = c.coop_bfs(rt.rt, dg.handle, rt._roots([0]), 1, lv, 0, plain)
    with pytest.raises(c.CoopError):
        c.coop_share_add(rt.rt, h, 1)              # sharer not running
    c.coop_share_start(rt.rt)
    try:
        with pytest.raises(c.CoopError):
            c.coop_share_add(rt.rt, h, 1)          # a plain launch cannot be resized
        with pytest.raises(c.CoopError):
            c.coop_share_start(rt.rt)              # already running
    finally:
        rcs, _ = c.coop_share_stop(rt.rt)
        rc, _ = c.coop_wait(h)
    assert rcs == 0 and rc == 0
    assert np.array_equal(lv.cpu().numpy().view(np.uint32), oracle.bfs(g, 0))
    dg.release()
