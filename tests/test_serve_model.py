"""The query server's host/device protocol, model-checked on the CPU
(oracle/serve_model.py): publish (record, owner entries, ticket end) ->
ticket draw -> owner lookup -> rank -> team barrier with members let go ->
last leaver's completion record -> slot reuse. Every interleaving keeps
tickets, slots and ranks consistent, never reuses a slot under a member and
completes every query; each planted mistake is caught."""
import pytest

from oracle.serve_model import ModelError, ServeModel

CASES = [(3, 1, [1, 2, 1], 2), (3, 2, [2, 1, 2], 2), (3, 2, [1, 1, 1, 1], 1), (4, 1, [3, 1], 3), (4, 2, [1, 3], 3)]


@pytest.mark.parametrize("W,S,teams,team_max", CASES)
def test_serve_protocol(W, S, teams, team_max):
    r = ServeModel(W, S, teams, team_max=team_max).explore()
    assert r["finals"] > 0


@pytest.mark.parametrize("mistake", ["early_end", "small_ring", "count_released", "no_gap_check"])
def test_planted_mistakes_are_caught(mistake):
    caught = False
    for W, S, teams, team_max in CASES:
        try:
            ServeModel(W, S, teams, team_max=team_max, mistake=mistake).explore()
        except ModelError:
            caught = True
            break
    assert caught, mistake
