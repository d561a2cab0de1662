"""Autotuner for the persistent trace launch.

Times candidate launch settings on the caller's own workload and keeps the
fastest: the launch tile (register budget = waves per SIMD, persistent
workgroups per compute unit), the ray queue (fetch threshold: idle lanes
before a wavefront takes new rays from the pool; shade threshold: finished
queries before it shades them) and the LDS traversal-stack depth per lane.
The search is coordinate descent from the library defaults (each parameter
in turn, the others held, two sweeps; repeated settings are timed once) or,
on request, the whole product.  Results are cached in a JSON file keyed by
(GPU architecture, log2 of the largest scene's triangle count, log2 of the
ray count), so a later call with a similar workload reuses the choice
without timing.

The cache lives at $RTAC_TUNE_CACHE, else ~/.cache/rtac/autotune.json.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Callable, Dict, List, Optional

import torch

DEFAULT_CANDIDATES = {
    "waves_per_simd": [4, 5],
    "blocks_per_cu": [0, 8],
    "fetch_threshold": [8, 16, 32],
    "shade_threshold": [8, 16, 32],
    "stack_depth": [8, 16, 32],
}
# library defaults (0 = the library's own choice), where coordinate descent starts
DEFAULT_START = {"waves_per_simd": 4, "blocks_per_cu": 0, "fetch_threshold": 16, "shade_threshold": 16,
                 "stack_depth": 16}


def cache_path() -> str:
    p = os.environ.get("RTAC_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "rtac", "autotune.json")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key_for(max_tris: int, n_rays: int) -> str:
    return "%s/m%d/n%d" % (_arch(), int(math.log2(max(1, max_tris))), int(math.log2(max(1, n_rays))))


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict[str, dict]) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(space: Optional[Dict[str, List[int]]] = None) -> List[dict]:
    space = space or DEFAULT_CANDIDATES
    names = sorted(space)
    return [dict(zip(names, vals)) for vals in itertools.product(*[space[n] for n in names])]


def _event_timer(run: Callable[[dict], None], repeats: int) -> Callable[[dict], float]:
    """Median of `repeats` event-timed runs after one warm-up run."""
    def timer(setting: dict) -> float:
        run(setting)
        torch.cuda.synchronize()
        times = []
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            run(setting)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return sorted(times)[len(times) // 2]
    return timer


def search(timer: Callable[[dict], float], space: Dict[str, List[int]], method: str = "coordinate",
           start: Optional[dict] = None, sweeps: int = 2, verbose: bool = False):
    """Best setting of `space` under `timer(setting) -> ms` (lower is better)
    and the table of timed settings.  "coordinate": from `start` (the first
    value of each parameter if absent), each parameter in turn over its
    values with the others held, `sweeps` times; "exhaustive": every
    combination.  Every distinct setting is timed once."""
    seen: Dict[tuple, float] = {}

    def time_of(setting: dict) -> float:
        k = tuple(sorted(setting.items()))
        if k not in seen:
            seen[k] = timer(setting)
            if verbose:
                print("autotune %s %.3f ms" % (setting, seen[k]), flush=True)
        return seen[k]

    if method == "exhaustive":
        best = min(candidates(space), key=time_of)
    elif method == "coordinate":
        best = {n: (start[n] if start and n in start and start[n] in space[n] else space[n][0]) for n in sorted(space)}
        best_ms = time_of(best)
        for _ in range(sweeps):
            changed = False
            for n in sorted(space):
                for v in space[n]:
                    trial = dict(best)
                    trial[n] = v
                    ms = time_of(trial)
                    if ms < best_ms:
                        best, best_ms, changed = trial, ms, True
            if not changed:
                break
    else:
        raise ValueError("method must be 'coordinate' or 'exhaustive'")
    table = sorted(((ms, dict(k)) for k, ms in seen.items()), key=lambda e: e[0])
    return dict(best), table


def tune(run: Callable[[dict], None], key: str, space: Optional[Dict[str, List[int]]] = None, repeats: int = 2,
         use_cache: bool = True, verbose: bool = False, method: str = "coordinate",
         timer: Optional[Callable[[dict], float]] = None) -> dict:
    """Return the fastest setting for `run(setting)` (which must launch the
    work on the current stream).  Each candidate is run once to warm up,
    then timed `repeats` times with events; the median decides (`timer`
    replaces that measurement)."""
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key]["setting"])
    space = space or DEFAULT_CANDIDATES
    best, table = search(timer or _event_timer(run, repeats), space, method=method, start=DEFAULT_START,
                         verbose=verbose)
    if use_cache:
        cache = _load()
        cache[key] = {"setting": best, "ms": table[0][0], "when": time.time(), "candidates": len(table),
                      "method": method}
        _store(cache)
    return best
