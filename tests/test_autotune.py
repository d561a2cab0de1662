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
    assert len(autotune.candidates()) == 2 * 2 * 3 * 3 * 3


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


def test_coordinate_descent_finds_a_separable_optimum_with_few_timings():
    from paper_1811_05784_amd import autotune
    space = autotune.DEFAULT_CANDIDATES
    want = {"waves_per_simd": 5, "blocks_per_cu": 8, "fetch_threshold": 32, "shade_threshold": 8, "stack_depth": 32}
    calls = []

    def timer(setting):
        calls.append(dict(setting))
        # separable cost with its minimum at `want`
        return 1.0 + sum(abs(space[n].index(setting[n]) - space[n].index(want[n])) for n in space)

    best, table = autotune.search(timer, space, start=autotune.DEFAULT_START)
    assert best == want
    assert len(calls) == len(table) == len({tuple(sorted(c.items())) for c in calls})   # each setting once
    assert len(calls) < len(autotune.candidates(space)) // 4
    small = {"waves_per_simd": [4, 5], "stack_depth": [8, 16]}
    ex, tab = autotune.search(lambda s: abs(s["waves_per_simd"] - 5) + abs(s["stack_depth"] - 16), small,
                              method="exhaustive")
    assert ex == {"waves_per_simd": 5, "stack_depth": 16} and len(tab) == 4


def test_tune_caches_the_search_result(tmp_path, monkeypatch):
    from paper_1811_05784_amd import autotune
    monkeypatch.setenv("RTAC_TUNE_CACHE", str(tmp_path / "t.json"))
    n = []
    best = autotune.tune(lambda s: None, "k", timer=lambda s: (n.append(1), 10.0 - s["stack_depth"] / 8)[1])
    assert best["stack_depth"] == 32 and n
    k = len(n)
    assert autotune.tune(lambda s: None, "k", timer=lambda s: n.append(1) or 0.0) == best and len(n) == k
    with pytest.raises(ValueError):
        autotune.search(lambda s: 0.0, {"a": [1]}, method="bogus")
