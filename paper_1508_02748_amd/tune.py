"""Autotuner for the batched sweep: walkers per workgroup, persistent-grid size and,
for batches smaller than one wavefront per CU, walkers per wavefront.

The launch shape changes neither the trajectory nor the tables (every random
number is addressed by walker and trial index), so candidates can be timed on
the plan's own state: the three device buffers are copied aside, each
candidate runs `intervals` profiled intervals (HIP events around the sweep
kernel), the buffers are restored after every candidate, and the fastest
shape is kept.  Choices are cached per (device, lattice-size mix, walker
count, interval) in a JSON file (``REWL_TUNE_CACHE``, default
``~/.cache/rewl_tune.json``).
"""
import json
import os

from . import FORM_BATCHED, Tuning

WG_CANDIDATES = (64, 128, 256)
GRID_CANDIDATES = (2, 3, 4, 5, 6, 8)
# a small batch can spread its walkers over more CUs (fewer lanes per wavefront)
WAVE_CANDIDATES = (32, 16, 8, 4, 2, 1)
SMALL_BATCH = 64 * 256


def _cache_path():
    return os.environ.get("REWL_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rewl_tune.json"))


def _key(plan):
    import torch
    name = torch.cuda.get_device_name(plan.device)
    sizes = {}
    for p in plan.problems:
        sizes[p.L] = sizes.get(p.L, 0) + p.n_windows * p.walkers_per_window
    mix = ",".join(f"{L}:{n}" for L, n in sorted(sizes.items()))
    split = getattr(plan.problems[0], "split", 0)
    return f"{name}|{mix}|{plan.n_walkers}|{plan.problems[0].interval}|split{split}"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def autotune(plan, intervals=1, candidates=None, use_cache=True, verbose=False):
    """Choose walkers_per_wg and grid_waves_per_cu for `plan` (batched form); returns the Tuning.

    The plan must have been initialised.  Its state after the call equals its
    state before it."""
    import torch

    if plan.tuning.form != FORM_BATCHED:
        raise ValueError("the autotuner times the batched form")
    path = _cache_path()
    key = _key(plan)
    base = plan.tuning
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            best = Tuning(form=FORM_BATCHED, walkers_per_wg=hit["wg"], graph_intervals=base.graph_intervals,
                          grid_waves_per_cu=hit["gw"], walkers_per_wave=hit.get("wpw", 0))
            plan.set_tuning(best)
            return best
    if candidates is None:
        candidates = [(wg, gw, 0) for wg in WG_CANDIDATES for gw in GRID_CANDIDATES]
        if plan.n_walkers < SMALL_BATCH:
            candidates += [(64, 0, wpw) for wpw in WAVE_CANDIDATES]
    candidates = [c if len(c) == 3 else (c[0], c[1], 0) for c in candidates]
    plan.stream.synchronize()
    saved = [b.clone() for b in plan.buffers]
    torch.cuda.synchronize(plan.device)
    results = []
    try:
        for wg, gw, wpw in candidates:
            t = Tuning(form=FORM_BATCHED, walkers_per_wg=wg, graph_intervals=base.graph_intervals,
                       grid_waves_per_cu=gw, profile=1, walkers_per_wave=wpw)
            plan.set_tuning(t)
            plan.run(intervals)
            ms = float(plan.sweep_times().mean())
            results.append((ms, wg, gw, wpw))
            if verbose:
                print(f"[tune] wg={wg} grid_waves_per_cu={gw} walkers_per_wave={wpw}: {ms:.3f} ms", flush=True)
            with torch.cuda.stream(plan.stream):
                for b, s in zip(plan.buffers, saved):
                    b.copy_(s)
            plan.stream.synchronize()
    finally:
        del saved
    ms, wg, gw, wpw = min(results)
    best = Tuning(form=FORM_BATCHED, walkers_per_wg=wg, graph_intervals=base.graph_intervals, grid_waves_per_cu=gw,
                  walkers_per_wave=wpw)
    plan.set_tuning(best)
    if use_cache:
        cache = _load_cache(path)
        cache[key] = {"wg": wg, "gw": gw, "wpw": wpw, "sweep_ms": ms}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best
