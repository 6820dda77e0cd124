"""Executable model of the cooperative-kernel scheduling semantics (CPU only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

This is a small transition system that restates, in plain Python, the
protocol the GPU runtime implements for the paper's resizing global barrier
with a ``query`` (the efficient scheduler-aware barrier of the paper's
scheduler-design section) and the semantics it must refine (the paper's
cooperative-kernel semantics section and the operational rules of its
Appendix A: Kill-No-Op, Kill, Fork, Barrier, Resizing-Barrier).

Every workgroup runs the level-synchronous traversal of the paper's
cooperative graph-traversal figure: claim frontier nodes, process them, then
one resizing barrier per level at which the last workgroup to arrive acts as
master (swaps frontiers, resets the output frontier, increments the level,
admits waiting joiners = fork, reads the scheduler target = query, and
releases; workgroups whose id is at or above the new count leave = kill).
The scheduler target T may change at any moment; joiner workgroups may
register at any moment.

``explore`` enumerates *every* interleaving of workgroup steps, target
changes and joiner arrivals (bounded by the given budgets) and checks, in
every reachable state:
  * 1 <= M <= N;
  * running workgroups hold distinct ids inside [0, M); when every running
    workgroup is waiting at the barrier they hold exactly {0, ..., M-1};
  * workgroup 0 never leaves before the kernel is done;
  * M changes only inside the barrier's master step, and each change is a
    fork of k in [0, N - M] new ids [M, M + k - 1] followed by a kill of the
    top ids (Resizing-Barrier = barrier, fork by 0, barrier, kill, barrier);
  * no deadlock: every non-final state has an enabled workgroup step;
  * every final state's output equals the plain BFS levels (the schedule
    that never kills or forks is a legal one, so all must agree with it).

With ``victims="any"`` the kill takes any W workgroups other than 0 (every
choice is explored) and renumbers the survivors densely in id order, the
kill-in-any-order variant of the paper's appendix. The master writes each
old id's new id tagged with the epoch; a waiter that sees the epoch advance
by one reads its entry in a separate step, and an entry of another epoch (it
was overwritten by a later barrier) means it was killed.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

INF = 0xFFFFFFFF

# workgroup program counters
UNSTARTED, WORK, PROC, ARRIVE, WAIT, POST, JWAIT, EXITED, COHORT = range(9)
PC_NAMES = ["UNSTARTED", "WORK", "PROC", "ARRIVE", "WAIT", "POST", "JWAIT", "EXITED", "COHORT"]


@dataclass(frozen=True)
class WG:
    pc: int = UNSTARTED
    logical: int = -1      # logical workgroup id, -1 until admitted
    seen: int = -1         # release epoch this workgroup last observed
    node: int = -1         # frontier node being processed
    arc: int = 0           # next arc of that node
    level: int = 0         # transmitted level
    joinslot: int = -1     # position in the joiner queue
    mseen: int = 0         # active count read together with `seen`
    rn: bool = False       # the observed release renumbered: read the new id
    grid: bool = True      # one of the launch's own workgroups (else of a joiner grid)
    ticket: int = -1       # start-up ticket (launch's own workgroups)


@dataclass(frozen=True)
class State:
    levels: Tuple[int, ...]
    frontier: Tuple[int, ...]       # input frontier of the current level
    out: Tuple[int, ...]            # output frontier being built
    claim: int                      # next frontier index to claim
    M: int
    Mnew: int                       # count published by the last master step
    epoch: int
    arrive: int
    level: int                      # transmitted level (master's copy)
    done: bool
    T: int                          # scheduler target (query)
    tickets: int                    # start-up registration counter
    joinq: Tuple[int, ...]          # physical ids waiting to be admitted
    admitted: Tuple[Tuple[int, int, int], ...]   # (physical id, logical id, epoch) per admission
    wgs: Tuple[WG, ...]
    t_changes: int                  # remaining scheduler target changes
    joiners_left: int               # remaining joiner workgroups the host may launch
    renum: Tuple[Tuple[int, int], ...] = ()    # per old id: (epoch, new id or -1)
    renum_epoch: int = -1           # epoch whose release carried a renumbering
    cohort: int = 0                 # tickets the first barrier admitted as ids 0 .. cohort-1


class ModelError(AssertionError):
    pass


class Model:
    """The transition system for one graph, source and launch size N."""

    def __init__(self, adj: Sequence[Sequence[int]], src: int, N: int, *,
                 t_changes: int = 1, joiners: int = 1, park_killed: bool = False,
                 t_values: Optional[Sequence[int]] = None, victims: str = "top"):
        self.adj = [tuple(a) for a in adj]
        self.n = len(adj)
        self.src = src
        self.N = N
        self.park = park_killed
        self.t_values = tuple(t_values) if t_values is not None else tuple(range(1, N + 1))
        self.init_t_changes = t_changes
        self.init_joiners = joiners
        if victims not in ("top", "any"):
            raise ValueError(victims)
        self.victims = victims

    # ------------------------------------------------------------ start
    def initial(self) -> State:
        levels = [INF] * self.n
        levels[self.src] = 0
        return State(levels=tuple(levels), frontier=(self.src,), out=(), claim=0,
                     M=1, Mnew=1, epoch=0, arrive=0, level=0, done=False, T=self.N,
                     tickets=0, joinq=(), admitted=(),
                     wgs=tuple(WG() for _ in range(self.N)),
                     t_changes=self.init_t_changes, joiners_left=self.init_joiners,
                     renum=tuple((-1, -1) for _ in range(self.N)), renum_epoch=-1)

    # ------------------------------------------------------ transitions
    def successors(self, s: State) -> List[Tuple[str, State]]:
        out: List[Tuple[str, State]] = []
        for i, w in enumerate(s.wgs):
            if w.pc == ARRIVE and s.arrive + 1 == s.M:
                for k, nxt in enumerate(self._master(s, i, w, all_choices=True)):
                    out.append((f"wg{i}:MASTER{k}", nxt))
                continue
            nxt = self._step_wg(s, i, w)
            if nxt is not None:
                out.append((f"wg{i}:{PC_NAMES[w.pc]}", nxt))
        if s.t_changes > 0 and not s.done:
            for t in self.t_values:
                if t != s.T:
                    out.append((f"T={t}", _replace(s, T=t, t_changes=s.t_changes - 1)))
        if s.joiners_left > 0:
            out.append(("launch-joiner", _replace(s, wgs=s.wgs + (WG(grid=False),),
                                                   joiners_left=s.joiners_left - 1)))
        return out

    def wg_enabled(self, s: State) -> bool:
        return any(self._step_wg(s, i, w) is not None for i, w in enumerate(s.wgs))

    def _set(self, s: State, i: int, w: WG, **kw) -> State:
        wgs = list(s.wgs)
        wgs[i] = w
        return _replace(s, wgs=tuple(wgs), **kw)

    def _step_wg(self, s: State, i: int, w: WG) -> Optional[State]:
        pc = w.pc
        if pc == UNSTARTED:
            # registration: the launch's own workgroups draw tickets; ticket
            # 0 is logical workgroup 0 (M starts at 1) and every later ticket
            # waits for the first release, whose master admitted the tickets
            # drawn before it as ids 0 .. cohort-1 (start-up admission); a
            # later ticket, and every workgroup of a joiner grid, is a
            # joiner, admitted at a barrier.
            if s.done:
                return self._set(s, i, _w(w, pc=EXITED))
            if not w.grid:
                return self._set(s, i, _w(w, pc=JWAIT, joinslot=len(s.joinq)), joinq=s.joinq + (i,))
            if s.tickets == 0:
                return self._set(s, i, _w(w, pc=WORK, logical=0, seen=s.epoch, level=s.level, ticket=0),
                                 tickets=1)
            return self._set(s, i, _w(w, pc=COHORT, ticket=s.tickets), tickets=s.tickets + 1)
        if pc == COHORT:
            if s.done:
                return self._set(s, i, _w(w, pc=EXITED))
            if s.epoch == 0:
                return None             # waiting for the first release
            if w.ticket < s.cohort:
                # a member of the first interval: the next barrier needs it,
                # so the first release is the one it sees
                if s.epoch != 1:
                    raise ModelError(f"start-up member saw epoch {s.epoch}")
                return self._set(s, i, _w(w, pc=POST, logical=w.ticket, seen=s.epoch, mseen=s.Mnew,
                                          level=s.level))
            return self._set(s, i, _w(w, pc=JWAIT, joinslot=len(s.joinq)), joinq=s.joinq + (i,))
        if pc == JWAIT:
            if s.done:
                return self._set(s, i, _w(w, pc=EXITED))
            for phys, lid, ep in s.admitted:
                if phys == i and w.joinslot >= 0 and s.epoch == ep:
                    # admitted at epoch ep: start right after the fork point
                    # with the transmitted state (level) of workgroup 0, once
                    # that epoch's release is visible
                    return self._set(s, i, _w(w, pc=POST, logical=lid, seen=s.epoch,
                                              mseen=s.Mnew, level=s.level, joinslot=-1))
            return None
        if pc == WORK:
            if s.claim < len(s.frontier):
                return self._set(s, i, _w(w, pc=PROC, node=s.frontier[s.claim], arc=0),
                                 claim=s.claim + 1)
            return self._set(s, i, _w(w, pc=ARRIVE))
        if pc == PROC:
            # one node's arcs in one step: claims are atomic test-and-set,
            # so each newly reached vertex has exactly one discoverer
            lv = list(s.levels)
            out = list(s.out)
            for u in self.adj[w.node]:
                if lv[u] == INF:
                    lv[u] = w.level + 1
                    out.append(u)
            return self._set(s, i, _w(w, pc=WORK, node=-1), levels=tuple(lv), out=tuple(out))
        if pc == ARRIVE:
            arrive = s.arrive + 1
            if arrive < s.M:
                return self._set(s, i, _w(w, pc=WAIT), arrive=arrive)
            return self._master(s, i, w, all_choices=False)[0]
        if pc == WAIT:
            if s.epoch != w.seen:
                # (epoch, count) are read as one word. An alive member is
                # needed by the next barrier, so it cannot miss an epoch: a
                # gap means this workgroup was killed at the epoch it missed.
                if s.epoch > w.seen + 1:
                    return self._set(s, i, _w(w, pc=POST, seen=s.epoch, mseen=-1))
                return self._set(s, i, _w(w, pc=POST, seen=s.epoch, mseen=s.Mnew,
                                          level=s.level, rn=s.renum_epoch == s.epoch))
            return None
        if pc == POST:
            if s.done:
                return self._set(s, i, _w(w, pc=EXITED, rn=False))
            if w.rn:
                # separate read of this id's entry: the barrier's own, or a
                # later one's if this workgroup was killed here
                ep, new = s.renum[w.logical]
                if ep != w.seen or new < 0:
                    return self._set(s, i, _w(w, rn=False, mseen=-1))
                return self._set(s, i, _w(w, rn=False, logical=new))
            if w.mseen < 0 or w.logical >= w.mseen:
                if w.logical == 0:
                    raise ModelError("workgroup 0 killed")
                if self.park:
                    return self._set(s, i, _w(w, pc=JWAIT, logical=-1, joinslot=len(s.joinq)),
                                     joinq=s.joinq + (i,))
                return self._set(s, i, _w(w, pc=EXITED, logical=-1))
            return self._set(s, i, _w(w, pc=WORK))
        return None   # EXITED

    def _master(self, s: State, i: int, w: WG, all_choices: bool) -> List[State]:
        """The last arrival runs the barrier's critical section while every
        other running workgroup waits: level bookkeeping, fork (admission of
        waiting joiners), query, and the kill decision. With victims="any"
        every choice of victims is a successor."""
        M = s.M
        members = sorted([x.logical for x in s.wgs if x.pc == WAIT and x.seen == s.epoch]
                         + [w.logical])
        if members != list(range(M)):
            raise ModelError(f"barrier membership {members} != 0..{M - 1}")
        # level bookkeeping (swap, reset, level++)
        frontier = s.out
        level = s.level + 1
        done = len(frontier) == 0
        # start-up admission (first barrier only): the tickets drawn so far,
        # at most the target, become ids 0 .. cohort-1
        cohort = s.cohort
        if s.epoch == 0 and not done:
            cohort = max(1, min(s.tickets, self.N, s.T))
            M = cohort
        # fork: k in [0, N - M], bounded by waiting joiners and the target
        k = 0 if done else min(len(s.joinq), self.N - M, max(0, s.T - M))
        # admission records persist (tagged with their epoch) so a slow
        # joiner cannot miss its own admission
        admitted = tuple(a for a in s.admitted if a[0] not in s.joinq[:k]) + \
            tuple((s.joinq[j], M + j, s.epoch + 1) for j in range(k))
        joinq = s.joinq[k:]
        M2 = M + k
        # query: W workgroups to give back, never workgroup 0
        W = 0 if done else min(max(0, M2 - s.T), M2 - 1)
        Mnew = M2 - W
        if not (0 < Mnew <= self.N) or not (0 <= k <= self.N - M):
            raise ModelError(f"bad resize M={M} k={k} W={W}")
        if W and k:
            raise ModelError("a barrier that admits joiners also kills")
        ne = s.epoch + 1
        base = dict(frontier=frontier, out=(), claim=0, level=level, done=done, arrive=0, M=Mnew,
                    Mnew=Mnew, epoch=ne, joinq=joinq, admitted=admitted, cohort=cohort)
        if self.victims == "top" or W == 0:
            s2 = _replace(s, **base)
            return [self._set(s2, i, _w(w, pc=POST, seen=ne, mseen=Mnew, level=level, rn=False))]
        from itertools import combinations
        result = []
        choices = list(combinations(range(1, M2), W))
        for victims in (choices if all_choices else choices[:1]):
            vs = set(victims)
            renum = list(s.renum)
            nxt = 0
            for old in range(M2):
                if old in vs:
                    renum[old] = (ne, -1)
                else:
                    renum[old] = (ne, nxt)
                    nxt += 1
            s2 = _replace(s, renum_epoch=ne, renum=tuple(renum), **base)
            # the master knows its own fate at once
            if w.logical in vs:
                result.append(self._set(s2, i, _w(w, pc=POST, seen=ne, mseen=-1, level=level, rn=False)))
            else:
                result.append(self._set(s2, i, _w(w, pc=POST, seen=ne, mseen=Mnew, level=level, rn=False,
                                                  logical=renum[w.logical][1])))
        return result

    # -------------------------------------------------------- invariants
    def check(self, s: State) -> None:
        if not s.done:
            if not (1 <= s.M <= self.N):
                raise ModelError(f"M out of range: {s.M}")
        running = [w for w in s.wgs if w.pc in (WORK, PROC, ARRIVE, WAIT, POST)]
        # a workgroup still waiting on an older epoch, or leaving after a
        # kill, is in transit: it has not yet observed the new count
        ids = [w.logical for w in running
               if not (w.pc == POST and (w.rn or w.mseen < 0 or w.logical >= w.mseen))
               and not (w.pc == WAIT and w.seen != s.epoch)]
        if len(ids) != len(set(ids)):
            raise ModelError(f"duplicate logical ids {ids}")
        if any(not (0 <= x < s.M) for x in ids) and not s.done:
            raise ModelError(f"id outside [0, M): {ids}, M={s.M}")
        if not s.done:
            if s.tickets > 0 and not any(w.logical == 0 and w.pc != EXITED for w in s.wgs):
                raise ModelError("workgroup 0 left before the end")
            waiting = [w for w in s.wgs if w.pc == WAIT and w.seen == s.epoch]
            if len(waiting) != s.arrive:
                raise ModelError(f"{len(waiting)} waiting but arrive counter {s.arrive}")

    def is_final(self, s: State) -> bool:
        return s.done and all(w.pc == EXITED for w in s.wgs) and s.joiners_left == 0


def _w(w: WG, **kw) -> WG:
    d = dict(w.__dict__)
    d.update(kw)
    return WG(**d)


def _replace(s: State, **kw) -> State:
    d = dict(s.__dict__)
    d.update(kw)
    return State(**d)


@dataclass
class ExploreResult:
    states: int
    finals: int
    outputs: set
    max_M_changes: int


def explore(model: Model, max_states: int = 2_000_000) -> ExploreResult:
    """Exhaustive search over every interleaving and scheduler choice."""
    init = model.initial()
    seen = {init}
    todo = deque([init])
    finals = 0
    outputs = set()
    while todo:
        s = todo.popleft()
        model.check(s)
        succ = model.successors(s)
        if model.is_final(s):
            finals += 1
            outputs.add(s.levels)
            continue
        if not model.wg_enabled(s) and not (s.done and s.joiners_left > 0):
            blocked = [PC_NAMES[w.pc] for w in s.wgs if w.pc != EXITED]
            raise ModelError(f"deadlock: {blocked}")
        for _, t in succ:
            if t not in seen:
                seen.add(t)
                if len(seen) > max_states:
                    raise ModelError("state budget exceeded")
                todo.append(t)
    return ExploreResult(states=len(seen), finals=finals, outputs=outputs, max_M_changes=0)


def random_run(model: Model, rng, max_steps: int = 1_000_000) -> State:
    """One seeded random schedule through the transition system."""
    s = model.initial()
    for _ in range(max_steps):
        model.check(s)
        if model.is_final(s):
            return s
        succ = model.successors(s)
        if not succ:
            raise ModelError("deadlock in random run")
        s = succ[rng.randrange(len(succ))][1]
    raise ModelError("random run did not terminate")
