"""GPU parity of the connected-components kernel, which is written only
against the programming-model calls of coop_device.hpp: its labels (the
smallest vertex id of each component) must equal the oracle's, element by
element, in plain and cooperative launches and under seeded random
kill/fork schedules (killed workgroups re-queue and are forked in again,
which only a correct resizing barrier, transmit block and rejoin survive)."""
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


def graphs(gg):
    return [gg.er(20000, 1.5, 4),                          # many components near the threshold
            gg.rmat(16, 8, seed=6),                       # one giant component and isolated vertices
            gg.grid(120, 150),                            # a long diameter: many rounds
            gg.disjoint_union(gg.disjoint_union(gg.path(3000), gg.empty(50)), gg.er(5000, 3, 8))]


@pytest.mark.parametrize("mode", ["plain", "coop", "coop_host"])
def test_cc_matches_oracle(rt, gg, mode):
    from paper_1707_01989_amd import coop as c
    if mode == "plain":
        opts = c.make_opts(c.COOP_MODE_PLAIN)
    elif mode == "coop":
        opts = c.make_opts(c.COOP_MODE_COOP)
    else:
        opts = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE)
    for g in graphs(gg):
        dg = rt.graph(g)
        rc, lab, st = rt.cc(dg, opts)
        say(f"cc {mode} {g.name}: rc={rc} rounds={st['barriers'] - 1} M={st['final_groups']}/{st['grid']}")
        assert rc == 0, c.coop_strerror(rc)
        assert np.array_equal(lab.cpu().numpy().view(np.uint32), oracle.cc(g)), g.name
        dg.release()


@pytest.mark.parametrize("seed", range(1, 7))
def test_cc_random_kill_fork(rt, gg, seed):
    """Seeded schedule: at each barrier the target moves with probability
    0.3 to a random value in [1, N]; surplus workgroups are killed (parked)
    and forked back in when the target rises."""
    from paper_1707_01989_amd import coop as c
    opts = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_RANDOM_SCHEDULE | c.COOP_F_PARK_KILLED,
                       sched_seed=seed, sched_p=0.3)
    kills = forks = 0
    for g in graphs(gg)[1:3]:
        dg = rt.graph(g)
        rc, lab, st = rt.cc(dg, opts)
        say(f"cc seed={seed} {g.name}: rounds={st['barriers'] - 1} kills={st['kills']} forks={st['forks']} "
            f"min M={st['min_groups']}")
        assert rc == 0, c.coop_strerror(rc)
        assert np.array_equal(lab.cpu().numpy().view(np.uint32), oracle.cc(g)), g.name
        kills += st["kills"]
        forks += st["forks"]
        dg.release()
    # a run of a few rounds may draw no kill; the grid's hundreds of rounds do
    assert kills > 0 and forks > 0


def test_cc_small_launch_and_joiners(rt, gg):
    """A launch of 3 workgroups of 64 threads (many vertices per thread) that
    a joiner grid grows under a host target."""
    from paper_1707_01989_amd import coop as c
    g = gg.grid(200, 200)
    dg = rt.graph(g)
    import torch
    lab = torch.empty(g.n, dtype=torch.int32, device="cuda")
    opts = c.make_opts(c.COOP_MODE_COOP, flags=c.COOP_F_HOST_SCHEDULE, num_groups=8, group_size=64)
    h = c.coop_cc(rt.rt, dg.handle, lab, opts)
    c.coop_set_target(h, 3)
    c.coop_set_target(h, 8)
    c.coop_fork_groups(h, 6)
    rc, st = c.coop_wait(h)
    say(f"cc joiners: rounds={st['barriers'] - 1} forks={st['forks']} kills={st['kills']}")
    assert rc == 0, c.coop_strerror(rc)
    assert np.array_equal(lab.cpu().numpy().view(np.uint32), oracle.cc(g))
    dg.release()
