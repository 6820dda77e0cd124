"""Executable model of the barrier's arrival by XCD (CPU only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The global barrier (the paper's master/slave barrier of its scheduler-design
section, with the Barrier and Resizing-Barrier rules of Appendix A) counts
arrivals in two tiers on the GPU: a workgroup adds 1 to the counter of its
XCD; the one that brings that counter to the XCD's member count resets it
and adds 1 to the top counter; the one that brings the top counter to the
number of XCDs with members is the master. Member counts per XCD are
published by the master with the release word and cached by every
workgroup, which reloads them only after a release that recounted them. An
interval right after joiners were admitted (whose XCDs are not recorded
yet) and the first interval arrive per workgroup on the top counter alone
(the flat interval). The same atomic adds that count also carry sums (a
BFS level's found count and degree sum): the XCD's last arriver passes the
sum its add returned up with its top-level add, and the master takes the
total from the value its own add returned.

This model restates that protocol one shared-memory step at a time (each
atomic add, store and load is its own transition) and ``explore`` runs every
interleaving of the workgroups' steps and of the scheduler's choices (which
joiners to admit and how many top ids to kill at each master step), checking
in every reachable state:
  * at most one master per barrier, and a master only when every member of
    the interval has arrived;
  * every XCD counter is back at 0 and the top counter at 0 whenever a
    release is published;
  * the per-XCD counts a workgroup uses equal the true member counts of its
    interval (a stale cache would make a counter wait forever or overshoot);
  * the sums the master receives are exactly the contributions of the
    interval's members (each contributes a bit of its own);
  * no deadlock: a state where some workgroup is not finished has an enabled
    step;
  * the final state: every barrier of the schedule was passed (the planned
    number of releases), and all workgroups left.

Plain mode is the special case with a fixed membership (every workgroup of
the grid, ids = block ids) and no scheduler choices. Memory is sequentially
consistent here: the model checks the counting protocol, not the GPU's
ordering of the operations (that comes from the waits, write-backs and
invalidations around the adds, which the kernels issue).
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, replace
from typing import Dict, List, Optional, Sequence, Tuple

FLAT = 1
DONE = 2
RENUM = 4

# workgroup program counters
(START, ENGINE, CHOOSE, LOADCNT, XADD, XRESET, XTOP, FLATADD, MASTER_RESET, MASTER, WAIT, JOINQ, JREC,
 EXITED) = range(14)


@dataclass(frozen=True)
class WG:
    pc: int = START
    xcd: int = 0                 # the XCD this workgroup runs on
    id: int = -1                 # logical id (-1 before admission)
    epoch: int = -1              # release epoch last seen (-1 before start)
    flags: int = 0               # flags of that release
    M: int = 0                   # members of the interval
    xm: int = 0                  # cached: members of this XCD
    xg: int = 0                  # cached: XCDs with members (0 = reload)
    last: bool = False           # this arrival made it the master
    carry: int = 0               # sums its arrival returned: its XCD's (by XCD), then the grand total


@dataclass(frozen=True)
class State:
    wgs: Tuple[WG, ...]
    xcnt: Tuple[int, ...]        # per-XCD arrival counters
    top: int                     # top arrival counter
    rel: Tuple[int, int, int]    # release word (epoch, M, flags)
    members: Tuple[int, ...]     # per-XCD member counts published for the interval
    groups: int                  # XCDs with members
    engine_of: Tuple[int, ...]   # XCD recorded per logical id (-1 = not yet)
    joinq: Tuple[int, ...]       # physical workgroups waiting to be admitted, in order
    admitted: Tuple[Tuple[int, int, int], ...]   # (physical, logical id, epoch)
    masters: Tuple[int, ...]     # epochs that have had a master (checked: no two)
    arrived: Tuple[int, ...]     # per physical workgroup: last epoch it arrived at (-1 none)
    xsum: Tuple[int, ...] = ()   # the sums riding on each XCD counter (same atomic as the count)
    topsum: int = 0              # ... and on the top counter
    hist: Tuple[int, ...] = ()   # M published at each epoch 1, 2, ...


class ModelError(AssertionError):
    pass


class ArrivalModel:
    """The protocol for `xcd_of` (the XCD of every physical workgroup of the
    grid), `barriers` barriers, and, in a cooperative launch, the scheduler
    choices `choices[e]` = list of (admit k, kill W) allowed at barrier e.

    Planted mistakes (each must be caught by ``explore``): "no_reset" (the
    XCD's last arriver does not reset its counter), "keep_cache" (counts are
    never reloaded after a recount), "no_flat" (the interval after an
    admission arrives by XCD although the joiners' XCDs are not recorded),
    "keep_sums" (the XCD's last arriver resets its count but not the sums
    riding on it)."""

    def __init__(self, xcd_of: Sequence[int], barriers: int, *, coop: bool = False,
                 joiner_xcds: Sequence[int] = (), choices: Optional[Sequence[Sequence[Tuple[int, int]]]] = None,
                 nxcd: Optional[int] = None, mistake: str = ""):
        self.grid = list(xcd_of)
        self.joiner_xcds = list(joiner_xcds)
        self.P = len(self.grid) + len(self.joiner_xcds)     # physical workgroups
        self.nx = nxcd if nxcd is not None else max(self.grid + self.joiner_xcds) + 1
        self.coop = coop
        self.B = barriers
        self.choices = [list(c) for c in choices] if choices is not None else None
        self.mistake = mistake
        self.N = self.P

    # ----------------------------------------------------------- start
    def initial(self) -> State:
        wgs = [WG(xcd=x) for x in self.grid] + [WG(pc=JOINQ, xcd=x) for x in self.joiner_xcds]
        if self.coop:
            # ticket 0 is workgroup 0, M = 1; the rest of the grid and the
            # joiner grid wait to be admitted (in physical order)
            wgs[0] = replace(wgs[0], pc=ENGINE, id=0, epoch=0, M=1)
            for p in range(1, len(self.grid)):
                wgs[p] = replace(wgs[p], pc=JOINQ)
            joinq = tuple(range(1, self.P))
            M0 = 1
        else:
            for p in range(len(self.grid)):
                wgs[p] = replace(wgs[p], pc=ENGINE, id=p, epoch=0, M=len(self.grid))
            joinq = ()
            M0 = len(self.grid)
        return State(wgs=tuple(wgs), xcnt=(0,) * self.nx, top=0, xsum=(0,) * self.nx, rel=(0, M0, 0),
                     members=(0,) * self.nx,
                     groups=0, engine_of=(-1,) * self.N, joinq=joinq, admitted=(), masters=(),
                     arrived=(-1,) * self.P)

    # ------------------------------------------------------- transitions
    def steps(self, s: State):
        """(label, next state) for every enabled step."""
        out = []
        for p, w in enumerate(s.wgs):
            for lab, ns in self._wg_steps(s, p, w):
                out.append((lab, ns))
        return out

    def _set(self, s: State, p: int, **kw) -> Tuple[WG, ...]:
        wgs = list(s.wgs)
        wgs[p] = replace(wgs[p], **kw)
        return tuple(wgs)

    def _wg_steps(self, s: State, p: int, w: WG):
        if w.pc == ENGINE:
            # record this workgroup's XCD for its id (registration / after admission)
            eo = list(s.engine_of)
            eo[w.id] = w.xcd
            yield ("engine", replace(s, engine_of=tuple(eo), wgs=self._set(s, p, pc=CHOOSE)))
        elif w.pc == CHOOSE:
            by_xcd = w.epoch != 0 and not (w.flags & FLAT)
            if self.mistake == "no_flat":
                by_xcd = w.epoch != 0
            arr = list(s.arrived)
            arr[p] = w.epoch
            ns = replace(s, arrived=tuple(arr))
            if by_xcd:
                yield ("choose", replace(ns, wgs=self._set(ns, p, pc=LOADCNT if w.xg == 0 else XADD)))
            else:
                yield ("choose", replace(ns, wgs=self._set(ns, p, pc=FLATADD)))
        elif w.pc == LOADCNT:
            yield ("loadcnt", replace(s, wgs=self._set(s, p, pc=XADD, xm=s.members[w.xcd], xg=s.groups)))
        elif w.pc == XADD:
            # one atomic: the count and this workgroup's contribution (the
            # bit 1 << p, so a sum names exactly who is in it)
            o = s.xcnt[w.xcd]
            osum = s.xsum[w.xcd]
            xc = list(s.xcnt)
            xc[w.xcd] = o + 1
            xs = list(s.xsum)
            xs[w.xcd] = osum + (1 << p)
            if o + 1 > w.xm:
                raise ModelError(f"XCD {w.xcd} counter passed its {w.xm} members (epoch {w.epoch})")
            nxt = XRESET if o + 1 == w.xm else WAIT
            yield ("xadd", replace(s, xcnt=tuple(xc), xsum=tuple(xs),
                                   wgs=self._set(s, p, pc=nxt, carry=osum + (1 << p))))
        elif w.pc == XRESET:
            xc = list(s.xcnt)
            xs = list(s.xsum)
            if self.mistake != "no_reset":
                xc[w.xcd] = 0
                if self.mistake != "keep_sums":
                    xs[w.xcd] = 0
            yield ("xreset", replace(s, xcnt=tuple(xc), xsum=tuple(xs), wgs=self._set(s, p, pc=XTOP)))
        elif w.pc == XTOP:
            o2 = s.top
            last = o2 + 1 == w.xg
            if o2 + 1 > w.xg:
                raise ModelError(f"top counter passed its {w.xg} XCD groups (epoch {w.epoch})")
            yield ("xtop", replace(s, top=o2 + 1, topsum=s.topsum + w.carry,
                                   wgs=self._set(s, p, pc=MASTER_RESET if last else WAIT,
                                                 carry=s.topsum + w.carry)))
        elif w.pc == FLATADD:
            old = s.top
            if old + 1 > w.M:
                raise ModelError(f"flat counter passed its {w.M} members (epoch {w.epoch})")
            last = old + 1 == w.M
            yield ("flatadd", replace(s, top=old + 1, topsum=s.topsum + (1 << p),
                                      wgs=self._set(s, p, pc=MASTER_RESET if last else WAIT,
                                                    carry=s.topsum + (1 << p))))
        elif w.pc == MASTER_RESET:
            yield ("mreset", replace(s, top=0, topsum=0, wgs=self._set(s, p, pc=MASTER)))
        elif w.pc == MASTER:
            yield from self._master(s, p, w)
        elif w.pc == WAIT:
            ep, M, fl = s.rel
            if ep != w.epoch:
                yield ("release", self._after_release(s, p, w))
        elif w.pc == JOINQ:
            ep, M, fl = s.rel
            adm = [a for a in s.admitted if a[0] == p]
            if adm:
                _, lid, aep = adm[0]
                if ep > aep:
                    # past its admission epoch: only a joiner that was not a
                    # member of that interval (admitted and killed at once) may be
                    if lid < s.hist[aep - 1]:
                        raise ModelError(f"joiner {p} (id {lid}) admitted at epoch {aep} missed it (release {ep})")
                    yield ("jgone", replace(s, wgs=self._set(s, p, pc=EXITED)))
                elif ep == aep:
                    if lid >= M:
                        # admitted and killed by the same master step: not a member
                        yield ("jkilled", replace(s, wgs=self._set(s, p, pc=EXITED)))
                    else:
                        yield ("joined", replace(s, wgs=self._set(s, p, pc=ENGINE, id=lid, epoch=ep, M=M,
                                                                 flags=fl, xm=0, xg=0)))
            elif fl & DONE:
                yield ("jleave", replace(s, wgs=self._set(s, p, pc=EXITED)))

    def _master(self, s: State, p: int, w: WG):
        ep = w.epoch
        if ep in s.masters:
            raise ModelError(f"two masters at epoch {ep}")
        # every member of the interval must have arrived
        members = [q for q, v in enumerate(s.wgs) if v.id >= 0 and v.epoch == ep and v.pc not in (JOINQ, EXITED)]
        for q in members:
            if s.arrived[q] != ep:
                raise ModelError(f"master at epoch {ep} before workgroup {q} arrived")
        # the sums the master's arrival returned are exactly the members' contributions
        if w.carry != sum(1 << q for q in members):
            raise ModelError(f"master at epoch {ep} got sums {w.carry:#x}, members "
                             f"{sum(1 << q for q in members):#x}")
        if any(c != 0 for c in s.xcnt) and self.mistake != "no_reset":
            raise ModelError(f"an XCD counter is not back at 0 at the master step of epoch {ep}: {s.xcnt}")
        ne = ep + 1
        done = ne > self.B
        opts = [(0, 0)]
        if self.coop and not done:
            opts = self.choices[ep] if self.choices is not None else [(0, 0)]
        for k, W in opts:
            k = min(k, len(s.joinq), self.N - w.M)
            M2 = w.M + k
            Wk = min(W, M2 - 1)
            Mn = M2 - Wk
            flags = DONE if done else 0
            adm = list(s.admitted)
            jq = list(s.joinq)
            for j in range(k):
                adm.append((jq[0], w.M + j, ne))
                jq.pop(0)
            if k and not done:
                flags |= FLAT
            members, groups = s.members, s.groups
            recount = (not done and k == 0 and (ep == 0 or (w.flags & FLAT) or Mn != w.M))
            if recount:
                cnt = [0] * self.nx
                for i in range(Mn):
                    x = s.engine_of[i]
                    if x < 0:
                        raise ModelError(f"recount at epoch {ep} reads the XCD of id {i}, not recorded")
                    cnt[x] += 1
                members, groups = tuple(cnt), sum(1 for c in cnt if c)
            ns = replace(s, rel=(ne, Mn, flags), members=members, groups=groups, joinq=tuple(jq),
                         admitted=tuple(adm), masters=s.masters + (ep,), hist=s.hist + (Mn,))
            # the master's own new member state
            nw = self._member_after(w, ne, Mn, flags)
            wgs = list(ns.wgs)
            wgs[p] = nw
            yield (f"master(k={k},W={Wk})", replace(ns, wgs=tuple(wgs)))

    def _counts_changed(self, w: WG, ne: int, Mn: int, flags: int) -> bool:
        if self.mistake == "keep_cache":
            return False
        if flags & (DONE | FLAT):
            return False
        return w.epoch == 0 or bool(w.flags & FLAT) or Mn != w.M or bool(flags & RENUM)

    def _member_after(self, w: WG, ne: int, Mn: int, flags: int) -> WG:
        alive = not (flags & DONE) and w.id < Mn
        xm, xg = w.xm, w.xg
        if self._counts_changed(w, ne, Mn, flags):
            xm, xg = 0, 0
        if not alive:
            return replace(w, pc=EXITED, epoch=ne, M=Mn, flags=flags, carry=0)
        return replace(w, pc=CHOOSE, epoch=ne, M=Mn, flags=flags, xm=xm, xg=xg, carry=0)

    def _after_release(self, s: State, p: int, w: WG) -> State:
        ep, M, fl = s.rel
        if ep != w.epoch + 1:
            # a member that sees the epoch jump was killed at the epoch it
            # missed (an alive one is needed by the next barrier); check it
            killed_M = s.hist[w.epoch]          # M published at epoch w.epoch + 1
            if w.id < killed_M:
                raise ModelError(f"workgroup {p} (id {w.id}) missed epoch {w.epoch + 1} while alive")
            return replace(s, wgs=self._set(s, p, pc=EXITED, epoch=ep, carry=0))
        return replace(s, wgs=self._set(s, p, **self._member_after(w, ep, M, fl).__dict__))

    # ------------------------------------------------------------ check
    def check_state(self, s: State):
        # cached counts used in an interval that arrives by XCD are the true ones
        ep, M, fl = s.rel
        if not (fl & (FLAT | DONE)) and ep > 0:
            true = [0] * self.nx
            for i in range(M):
                if s.engine_of[i] >= 0:
                    true[s.engine_of[i]] += 1
            for q, w in enumerate(s.wgs):
                if w.pc in (XADD,) and w.epoch == ep and w.xg:
                    if w.xm != true[w.xcd] or w.xg != sum(1 for c in true if c):
                        raise ModelError(f"workgroup {q} counts XCD {w.xcd} with {w.xm}/{w.xg} members/groups, "
                                         f"the interval has {true[w.xcd]}/{sum(1 for c in true if c)}")

    def explore(self, limit: int = 2_000_000) -> Dict[str, int]:
        s0 = self.initial()
        seen = {s0}
        q = deque([s0])
        finals = 0
        while q:
            s = q.popleft()
            self.check_state(s)
            nxt = self.steps(s)
            if not nxt:
                unfinished = [p for p, w in enumerate(s.wgs) if w.pc != EXITED]
                if unfinished:
                    raise ModelError(f"deadlock: workgroups {unfinished} stuck "
                                     f"({[ (s.wgs[p].pc, s.wgs[p].epoch) for p in unfinished]}), release {s.rel}, "
                                     f"xcnt {s.xcnt}, top {s.top}")
                if s.rel[0] != self.B + 1:
                    raise ModelError(f"finished after {s.rel[0]} releases, expected {self.B + 1}")
                finals += 1
                continue
            for _, ns in nxt:
                if ns not in seen:
                    if len(seen) >= limit:
                        raise ModelError("state limit reached")
                    seen.add(ns)
                    q.append(ns)
        return {"states": len(seen), "finals": finals}
