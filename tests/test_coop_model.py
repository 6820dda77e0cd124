"""Exhaustive check of the cooperative scheduling protocol on the CPU model.

The model restates the resizing-barrier protocol the GPU runtime uses (last
arrival acts as master: level bookkeeping, fork = admit waiting joiners,
query = read the scheduler target, kill = top ids leave) and explores every
interleaving of workgroup steps, target changes and joiner launches."""
import random

import pytest

from oracle import coop_model as cm

PATH4 = [[1], [0, 2], [1, 3], [2]]
STAR4 = [[1, 2, 3], [0], [0], [0]]
TRI = [[1, 2], [0, 2, 3], [0, 1], [1]]
BFS = {"path4": (0, 1, 2, 3), "star4": (0, 1, 1, 1), "tri": (0, 1, 1, 2)}
GRAPHS = {"path4": PATH4, "star4": STAR4, "tri": TRI}


@pytest.mark.parametrize("name", ["path4", "star4", "tri"])
@pytest.mark.parametrize("N,t_changes,joiners,park", [
    (1, 2, 1, False), (2, 2, 1, False), (2, 3, 0, True), (2, 2, 1, True), (3, 1, 0, True),
])
def test_exhaustive_no_deadlock_and_schedule_independent(name, N, t_changes, joiners, park):
    m = cm.Model(GRAPHS[name], 0, N, t_changes=t_changes, joiners=joiners, park_killed=park)
    r = cm.explore(m, max_states=400_000)
    assert r.finals > 0
    assert r.outputs == {BFS[name]}


def test_exhaustive_three_workgroups_with_exits():
    m = cm.Model(STAR4, 0, 3, t_changes=1, joiners=1, park_killed=False)
    r = cm.explore(m, max_states=400_000)
    assert r.outputs == {BFS["star4"]}


@pytest.mark.parametrize("seed", range(20))
def test_random_schedules_larger(seed):
    rng = random.Random(seed)
    n = 12
    adj = [[] for _ in range(n)]
    for _ in range(18):
        u, v = rng.randrange(n), rng.randrange(n)
        if u != v and v not in adj[u]:
            adj[u].append(v)
            adj[v].append(u)
    # plain BFS for the expected levels
    lv = [cm.INF] * n
    lv[0] = 0
    q = [0]
    for x in q:
        for y in adj[x]:
            if lv[y] == cm.INF:
                lv[y] = lv[x] + 1
                q.append(y)
    m = cm.Model(adj, 0, 6, t_changes=30, joiners=12, park_killed=bool(seed % 2))
    s = cm.random_run(m, rng)
    assert s.levels == tuple(lv)


class ReadsCountLate(cm.Model):
    """A planted protocol mistake: a waiting workgroup reads the epoch, and
    only later (separately) the active count. A killed workgroup that is slow
    can then see a later epoch's count and carry on with a stale id."""

    def _step_wg(self, s, i, w):
        if w.pc == cm.WAIT:
            if s.epoch != w.seen:
                return self._set(s, i, cm._w(w, pc=cm.POST, seen=s.epoch, mseen=-2, level=s.level))
            return None
        if w.pc == cm.POST and w.mseen == -2:
            w = cm._w(w, mseen=s.Mnew)
        return super()._step_wg(s, i, w)


def test_model_catches_planted_stale_count_race():
    m = ReadsCountLate(PATH4, 0, 2, t_changes=2, joiners=1, park_killed=False)
    with pytest.raises(cm.ModelError):
        cm.explore(m, max_states=400_000)
