"""Interleaving search over the joiner admission ring (CPU model in
oracle/ring_model.py): admitted slots belong to joiners that waited and read
the ids the master gave them, joiners that left are never counted, entry
indices are reused only after their previous slot was passed and read, and
no interleaving deadlocks -- including rings small enough to wrap, windows
that turn joiners away and slots the master passes unannounced. Planted
mistakes (the master admitting whatever a slot holds; a joiner announcing
over a newer slot's entry) are caught."""
import pytest

from oracle import ring_model as rm


@pytest.mark.parametrize("joiners,cap,n,window,barriers", [
    (2, 4, 2, 2, 3),
    (3, 4, 2, 2, 3),
    (3, 3, 1, 2, 3),
    (3, 2, 1, 1, 4),
])
def test_ring_exhaustive(joiners, cap, n, window, barriers):
    m = rm.RingModel(joiners=joiners, cap=cap, n=n, window=window, barriers=barriers, rooms=(0, n))
    r = rm.explore(m, max_states=1_000_000)
    assert r.finals > 0
    assert r.admitted_max == min(joiners, n * barriers)
    assert r.passed


def test_ring_exercises_wrap_and_window():
    m = rm.RingModel(joiners=3, cap=2, n=1, window=1, barriers=4, rooms=(0, 1))
    r = rm.explore(m, max_states=1_000_000)
    assert r.wrapped and r.window_leavers and r.passed


class _GreedyMaster(rm.RingModel):
    """The unbounded ring's mistake: the master counts a slot as admitted
    whatever its entry holds."""

    def _master_steps(self, s):
        for label, s2 in super()._master_steps(s):
            if label == "m:admit" and len(s2.master.valid) > len(s.master.valid):
                s2 = rm._rep(s2, master=rm._repm(s2.master, valid=s2.master.valid[:-1] + (True,)))
            yield label, s2


class _LapBlindJoiner(rm.RingModel):
    """A joiner that retries its compare-and-swap over whatever the entry
    holds, a newer slot's admission included."""

    def _joiner_steps(self, s, k, jn):
        if jn.pc == "cas" and jn.cur.slot > jn.slot:
            now = self._entry(s, jn.slot)
            if now == jn.cur:
                js = list(s.joiners)
                js[k] = rm._repj(jn, pc="wait")
                yield f"j{k}:announce", rm._rep(self._set_entry(s, jn.slot, rm.Entry(jn.slot, rm.WAITING)),
                                                joiners=tuple(js))
                return
        yield from super()._joiner_steps(s, k, jn)


def test_ring_model_catches_admitting_a_departed_joiner():
    m = _GreedyMaster(joiners=3, cap=4, n=2, window=2, barriers=3, rooms=(0, 2))
    with pytest.raises(rm.RingError):
        rm.explore(m, max_states=1_000_000)


def test_ring_model_catches_announcing_over_a_newer_slot():
    m = _LapBlindJoiner(joiners=3, cap=2, n=1, window=1, barriers=4, rooms=(0, 1))
    with pytest.raises(rm.RingError):
        rm.explore(m, max_states=1_000_000)
