"""Autotuner for the interaction launch shape.

For a given scene and precision it times whole steps for every supported
shape -- the row-split kernel with 1, 3 or 9 waves per 64-target chunk x 8,
16 or 64 targets per group, the group-per-wave kernel with 8, 16 or 64
targets per wave, the cooperative kernels with 8 or 16 -- keeps the fastest,
then times that shape with the workgroups taking chunks in runs of 1, 8 or 32
per XCD (interleaved repeats, median), sets the result in the library
(sph_set_tuning) and caches it in a JSON table keyed by the problem shape
(precision, particle count, grid).  A shape is (kernel, waves per chunk,
targets per group, XCD run); table entries without the fourth value mean run
1.  The table path comes from WCSPH_TUNE_CACHE (default: tune_table.json next
to this file, which holds the shapes measured on MI355X for the benchmark
workloads).
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

from . import lib

SPLITS = (1, 3, 9)
GROUPS = (8, 16, 64)
KERNEL_ROWS, KERNEL_GROUPS, KERNEL_COOP, KERNEL_COOP2 = 1, 2, 3, 4
#: (kernel, waves per chunk, targets per group)
SHAPES = tuple((KERNEL_ROWS, s, g) for s in SPLITS for g in GROUPS) + tuple(
    (KERNEL_GROUPS, 1, g) for g in GROUPS) + tuple(
    (k, 1, g) for k in (KERNEL_COOP, KERNEL_COOP2) for g in (8, 16))
CACHE = os.environ.get("WCSPH_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json"))


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


_state = {"fp64": (0, 0, 0, 0), "mixed": (0, 0, 0, 0)}
XCD_RUNS = (1, 8, 32)


def full_shape(shape):
    """(kernel, split, group, xcd_run) from a table entry: two-entry
    (split, group) entries mean the row-split kernel, three-entry ones run 1."""
    shape = tuple(int(v) for v in shape)
    if len(shape) == 2:
        shape = (KERNEL_ROWS,) + shape
    if len(shape) == 3:
        shape = shape + (1,)
    return shape


def apply(precision: str, shape) -> None:
    _state[precision] = full_shape(shape)
    f, m = _state["fp64"], _state["mixed"]
    lib.set_tuning(split_fp64=f[1], split_mixed=m[1], group_fp64=f[2], group_mixed=m[2],
                   kernel_fp64=f[0], kernel_mixed=m[0], xcd_run_fp64=f[3],
                   xcd_run_mixed=m[3])


def _pick_run(precision, shape, timed, repeats=3):
    """The XCD run (of XCD_RUNS) for `shape`: timed(run) returns seconds per
    step; interleaved repeats, the median of each."""
    import statistics
    ts = {r: [] for r in XCD_RUNS}
    for rep in range(repeats):
        # a different order each repeat: later steps of a developing flow cost more
        order = XCD_RUNS[rep % len(XCD_RUNS):] + XCD_RUNS[:rep % len(XCD_RUNS)]
        for r in order:
            apply(precision, tuple(shape[:3]) + (r,))
            ts[r].append(timed(r))
    med = {r: statistics.median(v) for r, v in ts.items()}
    best = min(med, key=med.get)
    apply(precision, tuple(shape[:3]) + (best,))
    return best, med


def tune(scene, precision: str = "mixed", steps: int = 30, warmup: int = 5,
         use_cache: bool = True, verbose: bool = False):
    """Pick (split, group) for (scene, precision); returns it (and applies it)."""
    import torch
    key = _key(precision, scene)
    tab = _load() if use_cache else {}
    if key in tab and "shape" in tab[key]:
        apply(precision, tab[key]["shape"])
        return full_shape(tab[key]["shape"])
    times = {}
    for shape in SHAPES:
        apply(precision, shape)
        sim = lib.Simulation(scene, precision)
        sim.run(warmup, -1.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps, -1.0, warmup)
        torch.cuda.synchronize()
        times[shape] = (time.perf_counter() - t0) / steps
        del sim
        if verbose:
            print(f"autotune {key} kernel={shape[0]} split={shape[1]} group={shape[2]}: "
                  f"{times[shape] * 1e3:.3f} ms/step", flush=True)
    best = min(times, key=times.get)

    def timed(run):
        sim = lib.Simulation(scene, precision)
        sim.run(warmup, -1.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps, -1.0, warmup)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps
    run, runs = _pick_run(precision, best, timed)
    best = tuple(best) + (run,)
    tab = _load()
    tab[key] = {"shape": list(best),
                "ms_per_step": {"%dx%dx%d" % k: v * 1e3 for k, v in times.items()},
                "xcd_run_ms_per_step": {str(r): v * 1e3 for r, v in runs.items()}}
    try:
        _save(tab)
    except OSError:
        pass
    return best


def tune_xcd_run(scene, precision: str = "mixed", steps: int = 30, warmup: int = 5):
    """Only the XCD run, for the table's (kernel, split, group) of this
    problem (tuned first if absent); updates the table entry."""
    import torch
    shape = tune(scene, precision)
    key = _key(precision, scene)

    def timed(run):
        sim = lib.Simulation(scene, precision)
        sim.run(warmup, -1.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps, -1.0, warmup)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps
    run, runs = _pick_run(precision, shape, timed)
    tab = _load()
    tab[key]["shape"] = list(shape[:3]) + [run]
    tab[key]["xcd_run_ms_per_step"] = {str(r): v * 1e3 for r, v in runs.items()}
    _save(tab)
    return tuple(tab[key]["shape"])


def cached_ensemble_shape(ens, precision: str = "mixed"):
    """The table's (kernel, split, group) for this batch, applied, or None."""
    tab = _load()
    key = f"ensemble:{precision}:n={ens.n}:inst={ens.ninst}"
    if key in tab and "shape" in tab[key]:
        apply(precision, tab[key]["shape"])
        return full_shape(tab[key]["shape"])
    return None


def tune_ensemble(ens, precision: str = "mixed", steps: int = 20, step0: int = 40,
                  use_cache: bool = True, verbose: bool = False):
    """(kernel, split, group) for a batch (lib.Ensemble), timed on the batch
    itself with the lagged fused step; cached like tune()."""
    import torch
    key = f"ensemble:{precision}:n={ens.n}:inst={ens.ninst}"
    tab = _load() if use_cache else {}
    if key in tab and "shape" in tab[key]:
        apply(precision, tab[key]["shape"])
        return full_shape(tab[key]["shape"])
    times = {}
    step = step0
    for shape in SHAPES:
        if shape[0] == KERNEL_ROWS and shape[1] == 9:
            continue  # nine waves per chunk never pays on batches this large
        apply(precision, shape)
        ens.run(2, -1.0, step, lib.RUN_LAGGED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.run(steps, -1.0, step + 2, lib.RUN_LAGGED)
        torch.cuda.synchronize()
        times[shape] = (time.perf_counter() - t0) / steps
        step += steps + 2
        if verbose:
            print(f"autotune {key} kernel={shape[0]} split={shape[1]} group={shape[2]}: "
                  f"{times[shape] * 1e3:.3f} ms/step", flush=True)
    best = min(times, key=times.get)
    clock = [step]

    def timed(run):
        ens.run(2, -1.0, clock[0], lib.RUN_LAGGED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.run(steps, -1.0, clock[0] + 2, lib.RUN_LAGGED)
        torch.cuda.synchronize()
        clock[0] += steps + 2
        return (time.perf_counter() - t0) / steps
    run, runs = _pick_run(precision, best, timed)
    best = tuple(best) + (run,)
    tab = _load()
    tab[key] = {"shape": list(best),
                "ms_per_step": {"%dx%dx%d" % k: v * 1e3 for k, v in times.items()},
                "xcd_run_ms_per_step": {str(r): v * 1e3 for r, v in runs.items()}}
    try:
        _save(tab)
    except OSError:
        pass
    return best


def tune_ensemble_xcd_run(ens, precision: str = "mixed", steps: int = 20, step0: int = 40):
    """Only the XCD run, for the table's (kernel, split, group) of this batch
    (tuned first if absent); updates the table entry."""
    import torch
    shape = tune_ensemble(ens, precision, steps=steps, step0=step0)
    key = f"ensemble:{precision}:n={ens.n}:inst={ens.ninst}"
    clock = [step0]

    def timed(run):
        ens.run(2, -1.0, clock[0], lib.RUN_LAGGED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.run(steps, -1.0, clock[0] + 2, lib.RUN_LAGGED)
        torch.cuda.synchronize()
        clock[0] += steps + 2
        return (time.perf_counter() - t0) / steps
    run, runs = _pick_run(precision, shape, timed)
    tab = _load()
    tab[key]["shape"] = list(shape[:3]) + [run]
    tab[key]["xcd_run_ms_per_step"] = {str(r): v * 1e3 for r, v in runs.items()}
    _save(tab)
    return tuple(tab[key]["shape"])
