"""The autotuner's cache file round-trips without a GPU: entries load, save
back identically, malformed files are refused whole."""
import pytest


@pytest.fixture
def coop():
    from paper_1707_01989_amd import coop as c
    return c


HEADER = "coop-tune-cache v1\n"
ENTRIES = [
    "gfx950 512 21949796 394870448 2097153 3 1  512 192 524288 24 1 512 512  181.250000\n",
    "gfx950 24 1086000 25200000 3000000 3 0  1024 0 1048576 32 0 2048 256  3.125000\n",
]


def test_cache_round_trip(coop, tmp_path):
    src = tmp_path / "in.txt"
    src.write_text(HEADER + "".join(ENTRIES))
    coop.coop_tune_cache_clear()
    assert coop.coop_tune_cache_load(str(src)) == 2
    out = tmp_path / "out.txt"
    assert coop.coop_tune_cache_save(str(out)) == 2
    lines = out.read_text().splitlines()
    assert lines[0] == HEADER.strip()
    norm = lambda l: l.split()
    assert sorted(map(norm, lines[1:])) == sorted(map(norm, [e.strip() for e in ENTRIES]))
    # loading the saved file again changes nothing
    assert coop.coop_tune_cache_load(str(out)) == 2
    coop.coop_tune_cache_clear()


@pytest.mark.parametrize("bad", [
    "not a cache\n" + ENTRIES[0],
    HEADER + "gfx950 512 1 2\n",                                   # short line
    HEADER + ENTRIES[0].replace(" 512 192 ", " 500 192 "),        # group size not a multiple of 64
    HEADER + ENTRIES[0].replace(" 512 192 ", " 512 4096 "),       # more workgroups than a launch holds
])
def test_cache_refuses_malformed(coop, tmp_path, bad):
    f = tmp_path / "bad.txt"
    f.write_text(bad)
    coop.coop_tune_cache_clear()
    with pytest.raises(coop.CoopError):
        coop.coop_tune_cache_load(str(f))
    out = tmp_path / "after.txt"
    assert coop.coop_tune_cache_save(str(out)) == 0      # nothing was taken


def test_cache_missing_file(coop, tmp_path):
    with pytest.raises(coop.CoopError):
        coop.coop_tune_cache_load(str(tmp_path / "missing.txt"))
