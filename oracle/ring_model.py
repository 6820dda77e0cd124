"""Executable model of the joiner admission ring (CPU only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Forks (the paper's request_fork) enter a resizable launch through a ring of
slots taken in arrival order. This model restates, one atomic memory step
at a time, the protocol the GPU runtime uses for that ring, so that a search
over interleavings can check it:

* a joiner takes slot s (an add on the tail), leaves at once if s lies a
  window or more ahead of the master's head, announces itself by turning the
  entry of s (kept at index s mod cap) into WAITING(s) with a
  compare-and-swap over an older slot's value only (its own slot's value
  means it was passed, a newer slot's that a lap went by while it stood
  still: it leaves), and may later give up with a compare-and-swap from
  WAITING(s) to WITHDRAWN(s); it learns it was admitted when the entry holds
  ADMIT(s, epoch, id), waits for that epoch's release and reads its final id;
* the master of a barrier with room admits the slots from its head on: it
  first reads each one and stops at the first slot taken since the previous
  barrier whose joiner has not announced itself yet (the cut); before the
  cut, a slot whose joiner waits becomes ADMIT(s, ...) by compare-and-swap,
  any other slot is closed (CONSUMED(s)) unless it is already withdrawn or
  closed; the admitted ones are renumbered densely; at a barrier without
  room it passes the leading withdrawn slots (a drain);
* a barrier cannot begin before every joiner admitted at the previous one
  has read its final id (they are members: the barrier waits for them).

``explore`` enumerates every interleaving (joiner steps, master steps, the
room of every barrier, every joiner's choice to give up) and checks in every
state that

* a slot the master counts as admitted belongs to a joiner that announced
  itself, never gave up and never left, and that joiner reads exactly the id
  the master gave it;
* no joiner that left (beyond the window, passed, or withdrawn) is counted;
* an entry index is written for a slot only after the master passed the
  index's previous slot and that slot's joiner, if admitted, read its id;
* no deadlock: a state with pending work has a step enabled.
"""
from __future__ import annotations

from dataclasses import dataclass, field

WAITING, WITHDRAWN, CONSUMED, ADMIT, STALE = "waiting", "withdrawn", "consumed", "admit", "stale"


@dataclass(frozen=True)
class Entry:
    slot: int
    tag: str
    epoch: int = -1
    ident: int = -1


@dataclass(frozen=True)
class Joiner:
    pc: str = "start"          # start, head, read, cas, wait, admitted, member, left_*
    slot: int = -1
    cur: Entry | None = None
    epoch: int = -1            # epoch of its admission
    ident: int = -1            # final id read


@dataclass(frozen=True)
class Master:
    pc: str = "idle"           # idle, classify, admit, renumber, drain
    barrier: int = 0           # barriers completed
    room: int = 0
    pre_tail: int = 0
    j: int = 0                 # slot cursor within the pass
    span: int = 0
    cut: int = 0
    cur: Entry | None = None   # entry read by the current compare-and-swap loop
    valid: tuple = ()          # per admitted slot: True if admitted
    drained: int = 0


@dataclass(frozen=True)
class State:
    tail: int
    head: int
    tail_prev: int
    entries: tuple
    joiners: tuple
    master: Master
    admitted: tuple = ()       # (slot, epoch, id) the master counted


class RingError(AssertionError):
    pass


@dataclass
class RingModel:
    joiners: int = 3           # joiner workgroups that will arrive
    cap: int = 4               # ring entries
    n: int = 2                 # launch limit: at most n slots pass per barrier
    window: int = 2            # joiners that may wait at once (cap - n)
    barriers: int = 4          # barriers the master runs
    rooms: tuple = (0, 2)      # room a barrier may have
    drain_min: int = 1         # queued slots before a room-less barrier drains

    def initial(self) -> State:
        return State(tail=0, head=0, tail_prev=0,
                     entries=tuple(Entry(-1, STALE) for _ in range(self.cap)),
                     joiners=tuple(Joiner() for _ in range(self.joiners)),
                     master=Master())

    # ------------------------------------------------------------ helpers
    def _set_entry(self, s: State, slot: int, e: Entry) -> State:
        i = slot % self.cap
        # the index's previous slot must have been passed by the master...
        if slot >= self.cap and slot - self.cap >= s.head:
            raise RingError(f"index {i} written for slot {slot} while slot {slot - self.cap} is still queued")
        # ...and a joiner admitted there must have read its final id
        for j in s.joiners:
            if j.slot != slot and j.slot >= 0 and j.slot % self.cap == i and j.pc == "admitted":
                raise RingError(f"index {i} written for slot {slot} before the joiner of slot {j.slot} "
                                "read its id")
        ents = list(s.entries)
        ents[i] = e
        return _rep(s, entries=tuple(ents))

    def _entry(self, s: State, slot: int) -> Entry:
        return s.entries[slot % self.cap]

    # -------------------------------------------------------------- steps
    def steps(self, s: State):
        """Yield (label, next_state) for every enabled atomic step."""
        for k, jn in enumerate(s.joiners):
            yield from self._joiner_steps(s, k, jn)
        yield from self._master_steps(s)

    def _joiner_steps(self, s: State, k: int, jn: Joiner):
        def put(**kw):
            js = list(s.joiners)
            js[k] = _repj(jn, **kw)
            return js

        if jn.pc == "start":
            yield f"j{k}:take", _rep(s, tail=s.tail + 1, joiners=tuple(put(pc="head", slot=s.tail)))
        elif jn.pc == "head":
            if jn.slot - s.head >= self.window:
                yield f"j{k}:full", _rep(s, joiners=tuple(put(pc="left_window")))
            else:
                yield f"j{k}:head", _rep(s, joiners=tuple(put(pc="read")))
        elif jn.pc == "read":
            yield f"j{k}:read", _rep(s, joiners=tuple(put(pc="cas", cur=self._entry(s, jn.slot))))
        elif jn.pc == "cas":
            if jn.cur.slot >= jn.slot:
                # our own slot's value (passed) or a newer slot's (a lap went by)
                if jn.cur.slot == jn.slot and jn.cur.tag != CONSUMED:
                    raise RingError(f"slot {jn.slot} holds {jn.cur} before its joiner announced itself")
                yield f"j{k}:passed", _rep(s, joiners=tuple(put(pc="left_passed")))
                return
            now = self._entry(s, jn.slot)
            if now == jn.cur:
                s2 = self._set_entry(s, jn.slot, Entry(jn.slot, WAITING))
                yield f"j{k}:announce", _rep(s2, joiners=tuple(put(pc="wait")))
            else:
                yield f"j{k}:reread", _rep(s, joiners=tuple(put(cur=now)))
        elif jn.pc == "wait":
            e = self._entry(s, jn.slot)
            if e.slot == jn.slot and e.tag == ADMIT:
                yield f"j{k}:seen", _rep(s, joiners=tuple(put(pc="admitted", epoch=e.epoch)))
            # give up (the target leaves no room, or the watchdog)
            if e == Entry(jn.slot, WAITING):
                s2 = self._set_entry(s, jn.slot, Entry(jn.slot, WITHDRAWN))
                yield f"j{k}:withdraw", _rep(s2, joiners=tuple(put(pc="left_withdrawn")))
        elif jn.pc == "admitted":
            if s.master.barrier >= jn.epoch:            # that epoch's release is out
                e = self._entry(s, jn.slot)
                if e.slot != jn.slot or e.tag != ADMIT or e.epoch != jn.epoch:
                    raise RingError(f"joiner of slot {jn.slot} reads {e} for its final id")
                yield f"j{k}:final", _rep(s, joiners=tuple(put(pc="member", ident=e.ident)))

    def _master_steps(self, s: State):
        m = s.master
        if m.pc == "idle":
            if m.barrier >= self.barriers:
                return
            # the barrier waits for the joiners admitted at the last one: they
            # are members, and a member arrives only after reading its id
            counted = {a[0] for a in s.admitted}
            if any(j.slot in counted and j.pc != "member" for j in s.joiners):
                return
            for room in self.rooms:
                ready = s.tail - s.head
                kmax = min(ready, room, self.n)
                if kmax:
                    yield f"m:begin(room={room})", _rep(s, master=_repm(m, pc="classify", room=room,
                                                                          pre_tail=s.tail, j=0, span=kmax,
                                                                          cut=kmax))
                else:
                    span = min(ready, self.n) if ready >= self.drain_min else 0
                    if span:
                        yield f"m:begin-drain", _rep(s, master=_repm(m, pc="drain", room=0, pre_tail=s.tail,
                                                                      j=0, span=span, drained=-1))
                    else:
                        yield f"m:publish-empty", self._publish(s, _repm(m, pre_tail=s.tail), 0, 0)
        elif m.pc == "classify":
            slot = s.head + m.j
            e = self._entry(s, slot)
            known = e.slot == slot and e.tag in (WAITING, WITHDRAWN, CONSUMED)
            cut = m.cut
            if not known and slot >= s.tail_prev:
                cut = min(cut, m.j)
            nm = _repm(m, j=m.j + 1, cut=cut)
            if m.j + 1 == m.span:
                nm = _repm(nm, pc="admit", j=0, valid=(), cur=None)
                if cut == 0:
                    yield "m:classify-end", self._publish(s, nm, 0, 0)
                    return
            yield "m:classify", _rep(s, master=nm)
        elif m.pc == "admit":
            slot = s.head + m.j
            cur = m.cur if m.cur is not None else None
            if cur is None:
                yield "m:admit-read", _rep(s, master=_repm(m, cur=self._entry(s, slot)))
                return
            now = self._entry(s, slot)
            done = None
            s2 = s
            if cur == Entry(slot, WITHDRAWN) or cur == Entry(slot, CONSUMED):
                done = False
            elif now != cur:
                yield "m:admit-retry", _rep(s, master=_repm(m, cur=now))
                return
            elif cur == Entry(slot, WAITING):
                s2 = self._set_entry(s, slot, Entry(slot, ADMIT, m.barrier + 1, -2))
                done = True
            else:
                s2 = self._set_entry(s, slot, Entry(slot, CONSUMED))
                done = False
            valid = m.valid + (done,)
            nm = _repm(m, j=m.j + 1, valid=valid, cur=None)
            if m.j + 1 == m.cut:
                nm = _repm(nm, pc="renumber", j=0)
            yield "m:admit", _rep(s2, master=nm)
        elif m.pc == "renumber":
            # every admitted slot gets its final id M + rank in one step each
            ranks = [i for i, v in enumerate(m.valid) if v]
            if m.j < len(ranks):
                j = ranks[m.j]
                slot = s.head + j
                e = self._entry(s, slot)
                base = len(s.admitted)
                s2 = self._set_entry(s, slot, Entry(slot, ADMIT, e.epoch, base + m.j))
                yield "m:renumber", _rep(s2, master=_repm(m, j=m.j + 1))
            else:
                adm = tuple((s.head + j, m.barrier + 1, len(s.admitted) + r) for r, j in enumerate(ranks))
                yield "m:publish", self._publish(_rep(s, admitted=s.admitted + adm), m, m.cut, 0)
        elif m.pc == "drain":
            slot = s.head + m.j
            e = self._entry(s, slot)
            drained = m.drained
            if drained < 0 and e != Entry(slot, WITHDRAWN):
                drained = m.j
            nm = _repm(m, j=m.j + 1, drained=drained)
            if m.j + 1 == m.span:
                d = m.span if drained < 0 else drained
                yield "m:drain-end", self._publish(s, nm, 0, d)
            else:
                yield "m:drain", _rep(s, master=nm)

    def _publish(self, s: State, m: Master, cut: int, drained: int) -> State:
        return _rep(s, head=s.head + cut + drained, tail_prev=m.pre_tail,
                    master=Master(pc="idle", barrier=m.barrier + 1))

    # ------------------------------------------------------------- checks
    def check(self, s: State) -> None:
        by_slot = {j.slot: j for j in s.joiners if j.slot >= 0}
        for slot, epoch, ident in s.admitted:
            j = by_slot.get(slot)
            if j is None or j.pc.startswith("left"):
                raise RingError(f"slot {slot} counted as admitted but its joiner is {j}")
            if j.pc == "member" and j.ident != ident:
                raise RingError(f"joiner of slot {slot} reads id {j.ident}, the master gave {ident}")
        if len({a[0] for a in s.admitted}) != len(s.admitted):
            raise RingError("a slot admitted twice")

    def final(self, s: State) -> bool:
        return s.master.pc == "idle" and s.master.barrier >= self.barriers and \
            all(j.pc in ("member", "wait", "start") or j.pc.startswith("left") for j in s.joiners)


def _rep(s: State, **kw) -> State:
    d = {f: getattr(s, f) for f in s.__dataclass_fields__}
    d.update(kw)
    return State(**d)


def _repj(j: Joiner, **kw) -> Joiner:
    d = {f: getattr(j, f) for f in j.__dataclass_fields__}
    d.update(kw)
    return Joiner(**d)


def _repm(m: Master, **kw) -> Master:
    d = {f: getattr(m, f) for f in m.__dataclass_fields__}
    d.update(kw)
    return Master(**d)


@dataclass
class RingResult:
    states: int = 0
    finals: int = 0
    admitted_max: int = 0
    window_leavers: bool = False
    passed: bool = False
    wrapped: bool = False
    outcomes: set = field(default_factory=set)


def explore(model: RingModel, max_states: int = 500_000) -> RingResult:
    """Every interleaving from the initial state; raises RingError on a
    violated property or a deadlock."""
    seen = set()
    stack = [model.initial()]
    r = RingResult()
    while stack:
        s = stack.pop()
        if s in seen:
            continue
        seen.add(s)
        if len(seen) > max_states:
            raise RuntimeError("state budget exhausted")
        model.check(s)
        nxt = list(model.steps(s))
        if not nxt:
            if not model.final(s):
                raise RingError(f"deadlock in {s}")
            r.finals += 1
            r.admitted_max = max(r.admitted_max, len(s.admitted))
            r.outcomes.add(tuple(j.pc for j in s.joiners))
        for _, s2 in nxt:
            stack.append(s2)
        r.window_leavers |= any(j.pc == "left_window" for j in s.joiners)
        r.passed |= any(j.pc == "left_passed" for j in s.joiners)
        r.wrapped |= s.tail > model.cap
    r.states = len(seen)
    return r
