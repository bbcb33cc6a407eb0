"""Host logic of the autotuner: the cache key, picking the fastest candidate,
and the JSON cache (hit without timing, forced re-tuning, other keys kept)."""
import json

import pytest

from paper_1105_5804_amd import tune


def test_candidates_cover_every_shape_and_schedule():
    assert len(tune.CANDIDATES) == 12
    assert {c[0] for c in tune.CANDIDATES} == {16, 32, 64, 128}
    assert {c[1] for c in tune.CANDIDATES} == {4, 8, 16}


def test_cache_key():
    assert tune.cache_key("gfx950", 16384, 16384, 3, "sweep") == "gfx950|16384x16384|q3|sweep"
    assert tune.cache_key("gfx950", 4096, 4096, 2, "sweep") != tune.cache_key("gfx950", 4096, 4096, 3, "sweep")
    assert tune.cache_key("gfx950", 64, 32, 2, "sweep") != tune.cache_key("gfx950", 32, 64, 2, "sweep")


def test_pick_fastest_and_ties():
    assert tune.pick({(16, 4): 3.0, (64, 8): 1.0, (128, 4): 2.0}) == (64, 8)
    assert tune.pick({(32, 4): 1.0, (64, 8): 1.0}) == (32, 4)
    with pytest.raises(ValueError):
        tune.pick({})


def test_tune_times_once_then_hits_cache(tmp_path):
    path = str(tmp_path / "t.json")
    calls = []

    def timer(c):
        calls.append(c)
        return {16: 5.0, 32: 3.0, 64: 1.5, 128: 2.0}[c[0]] + c[1] / 100.0

    e = tune.tune("k1", tune.CANDIDATES, timer, path=path)
    assert e["choice"] == [64, 4] and len(calls) == 12
    assert abs(e["ms"] - 1.54) < 1e-12
    again = tune.tune("k1", tune.CANDIDATES, timer, path=path)
    assert again == e and len(calls) == 12  # a cache hit times nothing
    forced = tune.tune("k1", tune.CANDIDATES, lambda c: 1.0 if c == (128, 16) else 9.0, force=True, path=path)
    assert forced["choice"] == [128, 16]
    tune.tune("k2", [(32, 8)], lambda c: 0.5, path=path)
    data = json.load(open(path))
    assert set(data) == {"k1", "k2"} and data["k1"]["choice"] == [128, 16]
    assert set(data["k1"]["timings"]) == {f"{th}/{mw}" for th, mw in tune.CANDIDATES}


def test_unreadable_cache_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert tune.load_cache(str(p)) == {}
    p.write_text("[1, 2]")
    assert tune.load_cache(str(p)) == {}
    assert tune.load_cache(str(tmp_path / "missing.json")) == {}


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("SWCCL_TUNE_CACHE", str(tmp_path / "x.json"))
    assert tune.cache_path() == str(tmp_path / "x.json")
