"""The barrier's arrival by XCD, model-checked on the CPU (oracle/arrival_model.py):
every interleaving of per-XCD adds, resets, top-counter adds, cached member
counts and flat intervals, for plain launches and for cooperative ones whose
master steps admit joiners or kill top ids, reaches the planned number of
barriers with exactly one master each and never deadlocks; planted mistakes
in the protocol are caught."""
import pytest

from oracle.arrival_model import ArrivalModel, ModelError

# what the master step can do in the kernels: admit k joiners (k <= T - M,
# so nothing is killed) or kill W top ids (nothing admitted)
CODE = [[(k, 0) for k in range(3)] + [(0, W) for W in (1, 2)]] * 4
# any combination, including admitting and killing at once (joiners then
# find they are not members and leave)
ANY = [[(k, W) for k in range(3) for W in range(3)]] * 4


@pytest.mark.parametrize("xcds", [[0, 1], [0, 0, 1], [0, 1, 1, 2], [0, 1, 0, 1], [1, 0, 2], [0, 0, 0]])
def test_plain_arrival(xcds):
    r = ArrivalModel(xcds, 5).explore()
    assert r["finals"] == 1


@pytest.mark.parametrize("grid,joiners", [([0, 1], [1]), ([0, 1, 0], []), ([0, 0], [1, 1]), ([1, 0], [0, 2]),
                                          ([0, 1, 2], [1])])
@pytest.mark.parametrize("choices", ["code", "any"])
def test_coop_arrival_with_admissions_and_kills(grid, joiners, choices):
    r = ArrivalModel(grid, 4, coop=True, joiner_xcds=joiners, choices=CODE if choices == "code" else ANY).explore()
    assert r["finals"] > 1


@pytest.mark.parametrize("mistake", ["no_reset", "keep_cache", "no_flat", "keep_sums"])
def test_planted_mistakes_are_caught(mistake):
    caught = False
    for grid, joiners, coop in (([0, 1, 0], [], False), ([0, 1], [1], True), ([0, 0], [1, 1], True)):
        try:
            ArrivalModel(grid, 4, coop=coop, joiner_xcds=joiners, choices=CODE, mistake=mistake).explore()
        except ModelError:
            caught = True
            break
    assert caught, mistake
