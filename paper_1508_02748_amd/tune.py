"""Autotuner for the batched form: launch shape of the sweep (walkers per
workgroup, persistent-grid size, walkers per wavefront), intervals per graph
launch, and -- before a plan exists -- the table layout.

Launch shape and graph length change neither the trajectory nor the tables
(every random number is addressed by walker and trial index), so candidates
are timed on the plan's own run, with no copy of its buffers: each candidate
runs `intervals` real intervals of the simulation with a HIP event pair around
every sweep kernel.  The candidates run in the order c1 .. cn and then
cn .. c1, and each is scored by the mean of its two timings; a drift of the
sweep time that is linear in the interval count (the sweep speeds up while
the tables fill) then adds the same amount to every score.  Afterwards the
plan has advanced by 2 n `intervals` intervals, exactly as it would have under
any fixed tuning.  The graph length (intervals per graph launch) is timed the
same way, by wall clock over graph replays, once the shape is chosen.

The table layout fixes the buffer sizes, so it is chosen before the plan is
created (`choose_layout`): each layout is timed on a probe plan of a few
replicas; under a memory budget the layout with the higher expected
throughput of the whole batch (replicas that fit / sweep time) is kept.

Choices are cached per (device, lattice-size mix, walker count, interval,
split, layout) in a JSON file (``REWL_TUNE_CACHE``, default
``~/.cache/rewl_tune.json``).
"""
import json
import os
import time

from . import FORM_BATCHED, LAYOUT_DENSE, LAYOUTS, Plan, Tuning, plan_bytes

WG_CANDIDATES = (64, 128, 256)
GRID_CANDIDATES = (2, 3, 4, 5, 6, 8)
# a batch below two wavefronts per SIMD can spread its walkers over more
# wavefronts (fewer lanes each), so that more SIMDs carry walkers
WAVE_CANDIDATES = (32, 16, 8, 4, 2, 1)
SPREAD_BELOW = 2 * 1024 * 64
GRAPH_CANDIDATES = (1, 4, 16)


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
    return (f"{name}|{mix}|{plan.n_walkers}|{plan.problems[0].interval}|split{split}"
            f"|layout{plan.tuning.table_layout}")


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _shape_candidates(plan):
    import torch
    cands = [(wg, gw, 0) for wg in WG_CANDIDATES for gw in GRID_CANDIDATES]
    if plan.n_walkers < SPREAD_BELOW:
        cands += [(64, 0, wpw) for wpw in WAVE_CANDIDATES if wpw * 1024 >= min(plan.n_walkers, 64 * 1024) // 4]
        # the fewest lanes per wavefront that still keep at most one wavefront per SIMD
        simds = 4 * torch.cuda.get_device_properties(plan.device).multi_processor_count
        fit = -(-plan.n_walkers // simds)
        if 1 <= fit < 64 and (64, 0, fit) not in cands:
            cands.append((64, 0, fit))
    return cands


def _with(base, **kw):
    d = dict(form=FORM_BATCHED, walkers_per_wg=base.walkers_per_wg, graph_intervals=base.graph_intervals,
             grid_waves_per_cu=base.grid_waves_per_cu, walkers_per_wave=base.walkers_per_wave,
             table_layout=base.table_layout, audit_shift=base.audit_shift, profile=0)
    d.update(kw)
    return Tuning(**d)


def autotune(plan, intervals=1, candidates=None, use_cache=True, verbose=False, graph_lengths=GRAPH_CANDIDATES):
    """Choose walkers_per_wg, grid_waves_per_cu, walkers_per_wave and graph_intervals for `plan`
    (batched form, initialised); returns the Tuning, which is also set on the plan.

    The plan keeps running while it is tuned (see the module notes); its results are those of any
    tuning.  `plan.tune_report` holds the timings."""
    import torch

    if plan.tuning.form != FORM_BATCHED:
        raise ValueError("the autotuner times the batched form")
    path = _cache_path()
    key = _key(plan)
    base = plan.tuning
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            best = _with(base, walkers_per_wg=hit["wg"], grid_waves_per_cu=hit["gw"],
                         walkers_per_wave=hit.get("wpw", 0), graph_intervals=hit.get("graph", 0))
            plan.set_tuning(best)
            plan.tune_report = {"cached": hit, "intervals_run": 0}
            return best
    if candidates is None:
        candidates = _shape_candidates(plan)
    candidates = [c if len(c) == 3 else (c[0], c[1], 0) for c in candidates]
    plan.stream.synchronize()
    torch.cuda.synchronize(plan.device)
    times = {c: [] for c in candidates}
    ran = 0
    for c in candidates + candidates[::-1]:
        wg, gw, wpw = c
        plan.set_tuning(_with(base, walkers_per_wg=wg, grid_waves_per_cu=gw, walkers_per_wave=wpw, profile=1))
        plan.run(intervals)
        ran += intervals
        times[c].append(float(plan.sweep_times().mean()))
    scores = sorted((sum(v) / len(v), c) for c, v in times.items())
    for ms, (wg, gw, wpw) in scores if verbose else ():
        print(f"[tune] wg={wg} grid_waves_per_cu={gw} walkers_per_wave={wpw}: {ms:.3f} ms", flush=True)
    ms, (wg, gw, wpw) = scores[0]
    shape = _with(base, walkers_per_wg=wg, grid_waves_per_cu=gw, walkers_per_wave=wpw)
    # intervals per graph launch, by wall clock over replays (palindromic order again)
    per_graph = {}
    for G in list(graph_lengths) + list(graph_lengths)[::-1]:
        plan.set_tuning(_with(shape, graph_intervals=G))
        plan.run(G)                               # captures the graph
        plan.stream.synchronize()
        t0 = time.perf_counter()
        plan.run(G)
        plan.stream.synchronize()
        per_graph.setdefault(G, []).append((time.perf_counter() - t0) / G * 1e3)
        ran += 2 * G
    graph_scores = sorted((sum(v) / len(v), G) for G, v in per_graph.items())
    if verbose:
        for gms, G in graph_scores:
            print(f"[tune] graph_intervals={G}: {gms:.3f} ms per interval", flush=True)
    best = _with(shape, graph_intervals=graph_scores[0][1])
    plan.set_tuning(best)
    plan.tune_report = {"sweep_ms": {f"{c[0]}/{c[1]}/{c[2]}": v for c, v in times.items()},
                        "graph_ms_per_interval": {str(G): v for G, v in per_graph.items()},
                        "chosen": {"wg": wg, "gw": gw, "wpw": wpw, "graph": graph_scores[0][1], "sweep_ms": ms},
                        "intervals_run": ran}
    if use_cache:
        cache = _load_cache(path)
        cache[key] = {"wg": wg, "gw": gw, "wpw": wpw, "graph": graph_scores[0][1], "sweep_ms": ms}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best


def choose_layout(problems_of, budget=None, probe_replicas=2, intervals=2, device="cuda:0", verbose=False,
                  max_replicas=None):
    """Table layout for a batch of replicas of one problem set; `problems_of(r)` gives the
    problems of r replicas.  Each layout in LAYOUTS that the problems allow (packed words need
    k_final <= 24) is timed on a probe plan of `probe_replicas` replicas over `intervals`
    intervals.  Without a memory budget the fastest layout wins.  With `budget` bytes, each
    layout's batch is as many replicas as fit, at most `max_replicas` (a batch beyond one
    wavefront per SIMD gains nothing), and the layout with the higher expected throughput
    (replicas / probe sweep time) wins, ties to the faster probe: a smaller layout can carry more
    walker chains.  Returns (layout, replicas or None, report).  Layouts do not change results."""
    import torch
    from . import RewlError
    report = {}
    for lay in LAYOUTS:
        try:
            per = plan_bytes(problems_of(1), lay)
        except RewlError as e:
            report[lay] = {"refused": str(e)}
            continue
        plan = Plan(problems_of(probe_replicas), Tuning(table_layout=lay, profile=1), device=device)
        plan.init()
        plan.run(1)
        plan.run(intervals)
        ms = float(plan.sweep_times().mean())
        plan.close()
        del plan
        torch.cuda.empty_cache()
        fit = None if budget is None else max(0, int(budget // per))
        if fit is not None and max_replicas is not None:
            fit = min(fit, int(max_replicas))
        report[lay] = {"probe_sweep_ms": ms, "bytes_per_replica": per, "replicas_fit": fit}
        if verbose:
            print(f"[tune] table_layout={lay}: probe sweep {ms:.3f} ms, {per / 2**30:.3f} GiB per replica, "
                  f"{fit} replicas fit", flush=True)
    ok = [lay for lay in LAYOUTS if "probe_sweep_ms" in report[lay]]
    if budget is None:
        return min(ok, key=lambda lay: report[lay]["probe_sweep_ms"]), None, report
    best = max(ok, key=lambda lay: (report[lay]["replicas_fit"] / report[lay]["probe_sweep_ms"],
                                    -report[lay]["probe_sweep_ms"]))
    if report[best]["replicas_fit"] < 1:
        return LAYOUT_DENSE, 1, report
    return best, report[best]["replicas_fit"], report
