"""Executable model of the query server's host/device protocol (CPU only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The server runs queries in one persistent launch (continuous batching).
The host publishes a query into a free slot: it writes the slot's request
record {query, team, first ticket}, the slot number into the ticket-owner
map for each of the team's tickets (a ring of `cap` entries), and then the
end of the published ticket range. An idle workgroup that sees a ticket
below that end draws it with compare-and-swap on the device's ticket
counter, looks up the slot in the owner map, reads the record and becomes
rank (ticket - first) of the query's team. The team meets at a barrier
whose master may release its top members to the scheduler (never member 0
and never below the team's floor); the members left after the query's last
barrier leave one by one, and the last of them writes the slot's
completion record, after which the host may reuse the slot.

``explore`` enumerates every interleaving of host steps (publish a queued
query into a free slot, poll a completion record) and device steps (one
shared-memory access each), with every choice of releases at the barrier,
and checks in every reachable state:
  * a drawn ticket's owner entry and the record it names belong to the
    query that ticket was published for, and the rank lies in [0, team)
    (the values the kernel then uses as indices);
  * a slot is reused only when no member of its previous query is in it;
  * the completion record is written once per query, by the last member,
    after every member that stays has passed the final barrier;
  * no deadlock while the launch holds at least team_max workgroups, and
    every query completes.

A member let go at a barrier may look at the slot's release word only after
the query has finished and the slot serves a later query: it must then
recognise the gap in epochs (an alive member cannot miss one) and leave,
instead of taking the later release for its own.

Planted mistakes (each must be caught): "early_end" (the host publishes the
ticket end before the owner entries), "small_ring" (the owner ring holds
fewer entries than tickets can be outstanding), "count_released" (the last
leaver counts the released members too), "no_gap_check" (a member let go
reads whatever release the slot shows).
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, replace
from typing import Dict, Optional, Sequence, Tuple

# workgroup program counters
IDLE, DRAW, OWNER, RECORD, ARRIVE, WAITREL, LEAVE, GONE = range(8)


@dataclass(frozen=True)
class WG:
    pc: int = IDLE
    t: int = -1          # ticket seen below the end / drawn
    slot: int = -1
    q: int = -1          # query (as read from the record)
    rank: int = -1
    team: int = 0
    epoch: int = 0       # the slot's barrier epoch when it joined


@dataclass(frozen=True)
class Slot:
    q: int = -1          # query in the slot (host's view: -1 free)
    rec: Tuple[int, int, int] = (-1, 0, 0)   # device-visible record (query, team, first)
    arrive: int = 0
    epoch: int = 0       # release epoch of the slot's barrier
    M: int = 0           # members after the last release
    left: int = 0        # leave counter
    done: int = -1       # completion record: the last query completed
    hist: Tuple[int, ...] = ()   # M published at each release epoch 1, 2, ... of the slot's barrier


@dataclass(frozen=True)
class State:
    wgs: Tuple[WG, ...]
    slots: Tuple[Slot, ...]
    owner: Tuple[int, ...]       # ticket-owner ring (slot per entry)
    end: int                     # published ticket end (device-visible)
    ticket: int                  # device ticket counter
    next_ticket: int             # host: next ticket to hand out
    queue: Tuple[int, ...]       # host: queries waiting for a slot
    completed: Tuple[int, ...]   # queries whose completion the host saw
    hstep: Tuple[int, int, int] = (-1, -1, 0)   # host publish in progress (query, slot, phase)


class ModelError(AssertionError):
    pass


class ServeModel:
    def __init__(self, workgroups: int, slots: int, teams: Sequence[int], *, team_max: int, cap: Optional[int] = None,
                 floor: int = 1, releases: bool = True, mistake: str = ""):
        self.W = workgroups
        self.S = slots
        self.teams = list(teams)
        self.team_max = team_max
        self.cap = cap if cap is not None else 2 * slots * team_max
        self.floor = floor
        self.releases = releases
        self.mistake = mistake
        if mistake == "small_ring":
            self.cap = max(1, team_max)

    def initial(self) -> State:
        return State(wgs=tuple(WG() for _ in range(self.W)), slots=tuple(Slot() for _ in range(self.S)),
                     owner=(-1,) * self.cap, end=0, ticket=0, next_ticket=0,
                     queue=tuple(range(len(self.teams))), completed=())

    # ------------------------------------------------------------ host
    def host_steps(self, s: State):
        q, sl, ph = s.hstep
        if q >= 0:
            # a publish in progress: record, owner entries, then the end
            team = self.teams[q]
            first = s.next_ticket
            if ph == 0:
                slots = list(s.slots)
                slots[sl] = replace(slots[sl], rec=(q, team, first), q=q)
                yield "h-record", replace(s, slots=tuple(slots), hstep=(q, sl, 1))
            elif ph == 1:
                if self.mistake == "early_end":
                    yield "h-end-early", replace(s, end=first + team, hstep=(q, sl, 2))
                else:
                    own = list(s.owner)
                    for k in range(team):
                        own[(first + k) % self.cap] = sl
                    yield "h-owner", replace(s, owner=tuple(own), hstep=(q, sl, 2))
            else:
                own = list(s.owner)
                if self.mistake == "early_end":
                    for k in range(team):
                        own[(first + k) % self.cap] = sl
                yield "h-end", replace(s, owner=tuple(own), end=first + team, next_ticket=first + team,
                                       hstep=(-1, -1, 0))
            return
        # poll completion records: a slot whose record shows its query done is free
        for i, slot in enumerate(s.slots):
            if slot.q >= 0 and slot.done == slot.q:
                for w in s.wgs:
                    if w.slot == i and w.q == slot.q and w.pc in (ARRIVE, LEAVE):
                        raise ModelError(f"slot {i} freed while a member of query {slot.q} is still in it")
                slots = list(s.slots)
                slots[i] = replace(slot, q=-1)
                yield f"h-done{slot.q}", replace(s, slots=tuple(slots), completed=tuple(sorted(s.completed + (slot.q,))))
        # publish the next queued query into a free slot (host's view)
        if s.queue:
            for i, slot in enumerate(s.slots):
                if slot.q < 0:
                    yield f"h-pub{s.queue[0]}", replace(s, queue=s.queue[1:], hstep=(s.queue[0], i, 0))
                    break

    # ---------------------------------------------------------- device
    def _set(self, s: State, p: int, **kw):
        wgs = list(s.wgs)
        wgs[p] = replace(wgs[p], **kw)
        return tuple(wgs)

    def _slot(self, s: State, i: int, **kw):
        slots = list(s.slots)
        slots[i] = replace(slots[i], **kw)
        return tuple(slots)

    def wg_steps(self, s: State, p: int, w: WG):
        if w.pc == IDLE:
            t = s.ticket
            if t < s.end:
                yield "see", replace(s, wgs=self._set(s, p, pc=DRAW, t=t))
            elif len(s.completed) == len(self.teams):
                yield "stop", replace(s, wgs=self._set(s, p, pc=GONE))
        elif w.pc == DRAW:
            if s.ticket == w.t:
                yield "draw", replace(s, ticket=w.t + 1, wgs=self._set(s, p, pc=OWNER))
            else:
                yield "lost", replace(s, wgs=self._set(s, p, pc=IDLE, t=-1))
        elif w.pc == OWNER:
            sl = s.owner[w.t % self.cap]
            if not (0 <= sl < self.S):
                raise ModelError(f"ticket {w.t}: owner entry {sl} is not a slot")
            yield "owner", replace(s, wgs=self._set(s, p, pc=RECORD, slot=sl))
        elif w.pc == RECORD:
            q, team, first = s.slots[w.slot].rec
            rank = w.t - first
            # the ticket must belong to this record's query
            tq = self._ticket_query(w.t)
            if q != tq:
                raise ModelError(f"ticket {w.t} of query {tq} reads the record of query {q} (slot {w.slot})")
            if not (0 <= rank < team) or team > self.team_max:
                raise ModelError(f"ticket {w.t}: rank {rank} outside its team of {team}")
            sl = s.slots[w.slot]
            yield "record", replace(s, wgs=self._set(s, p, pc=ARRIVE, q=q, rank=rank, team=team, epoch=sl.epoch))
        elif w.pc == ARRIVE:
            sl = s.slots[w.slot]
            if sl.epoch != w.epoch:
                raise ModelError(f"query {w.q} rank {w.rank} joined the slot at epoch {w.epoch}, "
                                 f"which moved to {sl.epoch} before it arrived")
            a = sl.arrive + 1
            if a < w.team:
                yield "arrive", replace(s, slots=self._slot(s, w.slot, arrive=a), wgs=self._set(s, p, pc=WAITREL))
            else:
                # master: release up to team - floor top members (never member 0)
                opts = [0]
                if self.releases:
                    # the scheduler keeps team_max workgroups in the launch
                    active = sum(1 for v in s.wgs if v.pc != GONE)
                    most = min(w.team - max(self.floor, 1), active - self.team_max)
                    opts = list(range(0, max(0, most) + 1))
                for rel in opts:
                    Mn = w.team - rel
                    ns = replace(s, slots=self._slot(s, w.slot, arrive=0, epoch=sl.epoch + 1, M=Mn,
                                                     hist=sl.hist + (Mn,)))
                    gone = w.rank >= Mn
                    yield f"master(rel={rel})", replace(ns, wgs=self._set(ns, p, pc=GONE if gone else LEAVE,
                                                                          epoch=sl.epoch + 1))
        elif w.pc == WAITREL:
            sl = s.slots[w.slot]
            if sl.epoch == w.epoch + 1:
                gone = w.rank >= sl.M
                yield "released", replace(s, wgs=self._set(s, p, pc=GONE if gone else LEAVE, epoch=sl.epoch))
            elif sl.epoch > w.epoch + 1:
                # the slot's barrier moved on more than once: an alive member
                # is needed by the next release, so this one was let go at
                # the epoch it missed (and the slot may already serve a later
                # query, whose release must not be taken for its own)
                if self.mistake == "no_gap_check":
                    if w.rank < sl.M:
                        raise ModelError(f"query {w.q} rank {w.rank} (let go at epoch {w.epoch + 1}) took the "
                                         f"release of epoch {sl.epoch} (M = {sl.M}) for its own")
                if w.rank < sl.hist[w.epoch]:
                    raise ModelError(f"query {w.q} rank {w.rank} missed epoch {w.epoch + 1} while a member")
                yield "let-go", replace(s, wgs=self._set(s, p, pc=GONE, epoch=sl.epoch))
        elif w.pc == LEAVE:
            sl = s.slots[w.slot]
            M = sl.M if self.mistake != "count_released" else w.team
            left = sl.left + 1
            if left > M:
                raise ModelError(f"slot {w.slot}: {left} leavers for {M} members")
            if left == M:
                if sl.done == w.q:
                    raise ModelError(f"query {w.q} completed twice")
                still = [v for q2, v in enumerate(s.wgs) if q2 != p and v.slot == w.slot and v.q == w.q
                         and (v.pc in (ARRIVE, LEAVE) or
                              (v.pc == WAITREL and v.rank < s.slots[w.slot].hist[v.epoch]))]
                if still:
                    raise ModelError(f"query {w.q} completed while members are still in it")
                ns = replace(s, slots=self._slot(s, w.slot, left=0, done=w.q))
            else:
                ns = replace(s, slots=self._slot(s, w.slot, left=left))
            yield "leave", replace(ns, wgs=self._set(ns, p, pc=IDLE, t=-1, slot=-1, q=-1, rank=-1, team=0))

    def _ticket_query(self, t: int) -> int:
        acc = 0
        for q, team in enumerate(self.teams):
            if acc <= t < acc + team:
                return q
            acc += team
        return -1

    def steps(self, s: State):
        out = list(self.host_steps(s))
        for p, w in enumerate(s.wgs):
            out.extend(self.wg_steps(s, p, w))
        return out

    def explore(self, limit: int = 3_000_000) -> Dict[str, int]:
        s0 = self.initial()
        seen = {s0}
        q = deque([s0])
        finals = 0
        while q:
            s = q.popleft()
            nxt = self.steps(s)
            if not nxt:
                if len(s.completed) != len(self.teams):
                    raise ModelError(f"deadlock: completed {s.completed}, queue {s.queue}, "
                                     f"workgroups {[(w.pc, w.q, w.rank) for w in s.wgs]}")
                finals += 1
                continue
            for _, ns in nxt:
                if ns not in seen:
                    if len(seen) >= limit:
                        raise ModelError("state limit reached")
                    seen.add(ns)
                    q.append(ns)
        return {"states": len(seen), "finals": finals}
