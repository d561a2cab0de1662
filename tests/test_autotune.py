"""Host logic of the launch autotuner: candidate enumeration and the JSON
cache (no GPU: the timed runner is replaced by a stub clock)."""
import json

import pytest


def test_candidates_cover_the_product():
    from paper_1811_05784_amd import autotune
    space = {"a": [1, 2], "b": [3, 4, 5]}
    c = autotune.candidates(space)
    assert len(c) == 6
    assert {tuple(sorted(x.items())) for x in c} == {(("a", i), ("b", j)) for i in (1, 2) for j in (3, 4, 5)}
    assert len(autotune.candidates()) == 36


def test_cache_roundtrip(tmp_path, monkeypatch):
    from paper_1811_05784_amd import autotune
    p = tmp_path / "sub" / "t.json"
    monkeypatch.setenv("RTAC_TUNE_CACHE", str(p))
    assert autotune.cache_path() == str(p)
    assert autotune._load() == {}
    autotune._store({"k": {"setting": {"a": 1}, "ms": 1.0}})
    assert json.loads(p.read_text())["k"]["setting"] == {"a": 1}
    assert autotune._load()["k"]["ms"] == 1.0
    p.write_text("not json")
    assert autotune._load() == {}
