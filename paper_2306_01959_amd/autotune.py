"""Autotuner for the interaction launch shape.

For a given scene and precision it times whole steps for every supported
split (waves per 64-target chunk: 1, 3, 9), keeps the fastest, sets it in the
library (sph_set_tuning) and caches the choice in a JSON file keyed by the
problem shape (precision, particle count, grid).  The cache path comes from
WCSPH_TUNE_CACHE (default: tune_cache.json next to this file).
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

from . import lib

SPLITS = (1, 3, 9)
CACHE = os.environ.get("WCSPH_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))


def _key(precision: str, scene) -> str:
    d = scene.params["dims"]
    return f"{precision}:n={scene.n}:dims={d[0]}x{d[1]}x{d[2]}"


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(tab: Dict[str, dict]) -> None:
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def current() -> Dict[str, int]:
    return dict(_state)


_state = {"fp64": 0, "mixed": 0}


def apply(precision: str, split: int) -> None:
    _state[precision] = int(split)
    lib.set_tuning(split_fp64=_state["fp64"], split_mixed=_state["mixed"])


def tune(scene, precision: str = "mixed", steps: int = 30, warmup: int = 5,
         use_cache: bool = True, verbose: bool = False) -> int:
    """Pick the split for (scene, precision); returns it (and applies it)."""
    import torch
    key = _key(precision, scene)
    tab = _load() if use_cache else {}
    if key in tab:
        apply(precision, tab[key]["split"])
        return tab[key]["split"]
    times = {}
    for split in SPLITS:
        apply(precision, split)
        sim = lib.Simulation(scene, precision)
        sim.run(warmup, -1.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps, -1.0, warmup)
        torch.cuda.synchronize()
        times[split] = (time.perf_counter() - t0) / steps
        del sim
        if verbose:
            print(f"autotune {key} split={split}: {times[split] * 1e3:.3f} ms/step", flush=True)
    best = min(times, key=times.get)
    apply(precision, best)
    tab = _load()
    tab[key] = {"split": best, "ms_per_step": {str(k): v * 1e3 for k, v in times.items()}}
    try:
        _save(tab)
    except OSError:
        pass
    return best


def tuned_split(scene, precision: str) -> Optional[int]:
    return _load().get(_key(precision, scene), {}).get("split")
