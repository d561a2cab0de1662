"""Autotuner for the persistent trace launch.

Times candidate launch settings (register budget = waves per SIMD,
persistent workgroups per compute unit, fetch and shade thresholds of the
wavefront loop) on the caller's own workload and keeps the fastest.  Results
are cached in a JSON file keyed by (GPU architecture, log2 of the largest
scene's triangle count, log2 of the ray count), so a later call with a
similar workload reuses the choice without timing.

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
}


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


def tune(run: Callable[[dict], None], key: str, space: Optional[Dict[str, List[int]]] = None, repeats: int = 2,
         use_cache: bool = True, verbose: bool = False) -> dict:
    """Return the fastest setting for `run(setting)` (which must launch the
    work on the current stream).  Each candidate is run once to warm up,
    then timed `repeats` times with events; the median decides."""
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key]["setting"])
    best, best_ms, table = None, float("inf"), []
    for setting in candidates(space):
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
        ms = sorted(times)[len(times) // 2]
        table.append((ms, setting))
        if verbose:
            print("autotune %s %.3f ms" % (setting, ms), flush=True)
        if ms < best_ms:
            best, best_ms = setting, ms
    if use_cache:
        cache = _load()
        cache[key] = {"setting": best, "ms": best_ms, "when": time.time(), "candidates": len(table)}
        _store(cache)
    return dict(best)
