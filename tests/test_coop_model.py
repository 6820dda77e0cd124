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


# ---------------------------------------------- kill in any order (renumbering)

@pytest.mark.parametrize("name,N,t_changes,joiners,park", [
    ("path4", 2, 2, 1, False), ("tri", 2, 2, 1, False), ("path4", 3, 2, 0, True), ("tri", 3, 2, 0, True),
    ("star4", 3, 1, 1, False), ("star4", 3, 2, 1, True),
])
def test_any_victims_exhaustive(name, N, t_changes, joiners, park):
    """Every choice of victims, every interleaving: no deadlock, distinct
    dense ids at every barrier, output equal to the plain BFS."""
    m = cm.Model(GRAPHS[name], 0, N, t_changes=t_changes, joiners=joiners, park_killed=park,
                 t_values=range(1, N + 1), victims="any")
    r = cm.explore(m, max_states=800_000)
    assert r.finals > 0
    assert r.outputs == {BFS[name]}


@pytest.mark.parametrize("seed", range(10))
def test_any_victims_random_schedules(seed):
    rng = random.Random(100 + seed)
    n = 10
    adj = [[] for _ in range(n)]
    for _ in range(16):
        u, v = rng.randrange(n), rng.randrange(n)
        if u != v and v not in adj[u]:
            adj[u].append(v)
            adj[v].append(u)
    lv = [cm.INF] * n
    lv[0] = 0
    q = [0]
    for x in q:
        for y in adj[x]:
            if lv[y] == cm.INF:
                lv[y] = lv[x] + 1
                q.append(y)
    m = cm.Model(adj, 0, 5, t_changes=25, joiners=10, park_killed=bool(seed % 2), victims="any")
    s = cm.random_run(m, rng)
    assert s.levels == tuple(lv)


class ReadsAnyRenumEntry(cm.Model):
    """A planted mistake: a waiter takes its entry of the renumbering table
    without checking that it belongs to the epoch it observed. A slow victim
    can then pick up a later barrier's id and run with a duplicate."""

    def _step_wg(self, s, i, w):
        if w.pc == cm.POST and w.rn and not s.done:
            ep, new = s.renum[w.logical]
            if new < 0:
                return self._set(s, i, cm._w(w, rn=False, mseen=-1))
            return self._set(s, i, cm._w(w, rn=False, logical=new))
        return super()._step_wg(s, i, w)


def _scripted(model, log=None):
    """Drive the model through one schedule: three workgroups; at the first
    barrier with all three the target drops to 2 and id 1 is the victim,
    which then stalls before reading its entry; the target goes back to 3
    (the joiner is admitted as id 2), then to 2 again with victim 2, so old
    id 1 is rewritten as a survivor's entry. Returns the final state."""
    s = model.initial()
    stage, victim, rr = 0, None, 0
    for _ in range(100_000):
        model.check(s)
        if model.is_final(s):
            return s
        succ = dict(model.successors(s))
        pick = None
        if stage == 0 and s.M == 3 and "T=2" in succ:
            pick, stage = "T=2", 1
        elif stage == 1:
            for lab in succ:
                if lab.endswith(":MASTER0"):
                    victim = [i for i, w in enumerate(s.wgs) if w.logical == 1][0]
                    pick, stage = lab, 2
        elif stage == 2 and s.wgs[victim].pc == cm.POST and "launch-joiner" in succ:
            pick, stage = "launch-joiner", 3
        elif stage == 3 and "T=3" in succ and len(s.wgs) > 3 and s.wgs[3].pc == cm.JWAIT:
            pick, stage = "T=3", 4
        elif stage == 4 and s.M == 3 and "T=2" in succ:
            pick, stage = "T=2", 5
        elif stage == 5:
            for lab in succ:
                if lab.endswith(":MASTER1"):
                    pick, stage = lab, 6
        if pick is not None and log is not None:
            log.append((stage, pick, s.epoch, s.M, [(cm.PC_NAMES[w.pc], w.logical) for w in s.wgs]))
        if pick is None:
            # round robin over the workgroups that may step
            cand = [lab for lab in succ if lab.startswith("wg")
                    and not (victim is not None and lab == f"wg{victim}:POST" and stage < 6)]
            if cand:
                nw = len(s.wgs)
                cand.sort(key=lambda lab: (int(lab[2:lab.index(":")]) - rr) % nw)
                pick = cand[0]
                rr += 1
        if pick is None:
            pick = next(iter(succ))
        s = succ[pick]
    raise AssertionError("script did not finish")


def test_model_scripted_victim_reads_stale_entry():
    P8 = [[1], [0, 2], [1, 3], [2, 4], [3, 5], [4, 6], [5, 7], [6]]
    kw = dict(t_changes=3, joiners=1, park_killed=False, t_values=(2, 3), victims="any")
    # the protocol: the stalled victim sees an entry of a later epoch and leaves
    final = _scripted(cm.Model(P8, 0, 3, **kw))
    assert final.levels == tuple(range(8))
    # the planted mistake: it takes that entry as its new id (a duplicate)
    with pytest.raises(cm.ModelError):
        _scripted(ReadsAnyRenumEntry(P8, 0, 3, **kw))


class CohortRecorder(cm.Model):
    """Records the largest start-up admission the search reaches."""
    largest = 0

    def check(self, s):
        CohortRecorder.largest = max(CohortRecorder.largest, s.cohort)
        super().check(s)


def test_startup_admission_is_explored():
    """The first barrier admits every ticket drawn before it (ids 0 ..
    cohort-1); the search reaches admissions of the whole launch."""
    CohortRecorder.largest = 0
    m = CohortRecorder(STAR4, 0, 3, t_changes=1, joiners=1, park_killed=False)
    r = cm.explore(m, max_states=400_000)
    assert r.outputs == {BFS["star4"]}
    assert CohortRecorder.largest == 3


class CohortIgnoresBound(cm.Model):
    """A planted mistake: a start-up workgroup takes its ticket as its id
    even when the first barrier did not admit it (ticket >= cohort)."""

    def _step_wg(self, s, i, w):
        if w.pc == cm.COHORT and s.epoch >= 1 and w.ticket >= s.cohort and not s.done:
            return self._set(s, i, cm._w(w, pc=cm.POST, logical=w.ticket, seen=s.epoch, mseen=s.Mnew,
                                         level=s.level))
        return super()._step_wg(s, i, w)


def test_model_catches_startup_member_beyond_admission():
    # a ticket drawn after the first barrier would share its id with the
    # joiner-grid workgroup admitted there
    m = CohortIgnoresBound(PATH4, 0, 3, t_changes=1, joiners=1, park_killed=False)
    with pytest.raises(cm.ModelError):
        cm.explore(m, max_states=400_000)
