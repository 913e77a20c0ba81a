"""Throughput of two-dimensional replica-exchange Wang-Landau sampling on one MI355X.

One step = one REWL interval over the whole batch: X Wang-Landau trials per
walker (Eq. 1 random walk in (E, M)), the flatness check and ln f reduction,
and one exchange round between adjacent windows (Eq. 2).

Headline workload: the 64x64 periodic Ising REWL problem (64 energy windows
with 3/4 overlap, full M range, 4 walkers per window, ln f from 1 to 2^-20,
80 % flatness, exchange every 10^5 trials, random initial spins) replicated
with independent seeds, as many replicas as the device memory holds, so that
the GPU carries as many walker chains as it can.  Inputs are synthetic (seeded
spins); every table and configuration is resident in HBM before the timed
region.  The 16x16 workload (8 windows x 4 walkers, X = 10^4) and the 32x32
plus mixed-L batch are measured next to it as extra keys.

Prints one JSON line: batched throughput (value), the plain
one-launch-per-window form on one problem next to the batched form on the
same problem (same trials, so the same final ln f), the roofline of the sweep
kernel (timed with HIP events around each of its launches) and the CPU oracle
on the host's cores (one core and all of them).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/sec on 1 MI355X (batched vs plain) at equal final ln f"
# One REWL problem of each measured configuration; the 64x64 problem is the
# one the throughput is quoted on.
C2 = dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=20, flat=(4, 5), interval=10_000)
C3 = dict(L=32, n_windows=16, overlap=(3, 4), walkers_per_window=8, k_final=24, flat=(4, 5), interval=10_000)
C4 = dict(L=64, n_windows=64, overlap=(3, 4), walkers_per_window=4, k_final=20, flat=(4, 5), interval=100_000)
# A mixed batch of lattice sizes with uneven window counts, run in the same
# launches as the 32x32 problems.
MIXED = [dict(C3, L=L, n_windows=nw) for L, nw in ((8, 2), (12, 4), (16, 8), (24, 12), (32, 16))]
# table layout of the extra workloads measured next to the headline (their launch shape is
# autotuned on the plan itself); their default replica counts fill the 1024 SIMDs with one
# wavefront of 64 walkers each (c2: two tiles of walkers per wavefront)
EXTRA_LAYOUT = {"c2": 0, "c3mix": 0}
# name -> (problems of one replica, default replica count, description)
WORKLOADS = {
    "c2": ([C2], 4096, "16x16 periodic Ising 2D-REWL (8 windows x 4 walkers, overlap 3/4, ln f 1 -> 2^-20, "
                       "80% flat, exchange every 10^4 trials)"),
    "c3": ([C3], 512, "32x32 periodic Ising 2D-REWL (16 windows x 8 walkers, overlap 3/4, ln f 1 -> 2^-24, "
                      "80% flat, exchange every 10^4 trials)"),
    "c3mix": ([C3] + MIXED, 141, "32x32 periodic Ising 2D-REWL (16 windows x 8 walkers, overlap 3/4, ln f 1 -> "
                                 "2^-24, 80% flat, exchange every 10^4 trials) plus a mixed batch of L in "
                                 "{8,12,16,24,32} with 2/4/8/12/16 windows x 8 walkers, all in the same launches"),
    "c4": ([C4], 0, "64x64 periodic Ising 2D-REWL (64 windows x 4 walkers, overlap 3/4, ln f 1 -> 2^-20, "
                    "80% flat, exchange every 10^5 trials)"),
}
# replicas 0 = as many as fit in the device memory (leaving MEM_SPARE bytes)
MEM_SPARE = 12 << 30


# Whole runs to the end (--full-run): the 4x4 serial 2D-WL problem, or the 8x8 REWL problem of the
# paper's experiments (3 windows with overlap 1/2 x 3 walkers, ln f 1 -> 2^-20).
FULL_RUN = {
    "c1": (dict(L=4, n_windows=1, overlap=(3, 4), walkers_per_window=1, k_final=16, flat=(4, 5), interval=10_000),
           "4x4 periodic Ising serial 2D-WL (1 window x 1 walker, ln f 1 -> 2^-16, 80% flat, flatness check every "
           "10^4 trials), run to the end"),
    "p8": (dict(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=3, k_final=20, flat=(4, 5), interval=10_000),
           "8x8 periodic Ising 2D-REWL (3 windows x 3 walkers, overlap 1/2, ln f 1 -> 2^-20, 80% flat, exchange "
           "every 10^4 trials), run to the end"),
}


def full_run(R, torch, replicas, which="c1"):
    """Whole runs to the final ln f (Sec. 2): one problem once in the plain form, once in the batched
    form (same final state, so the same final ln f), and `replicas` independent copies in one
    batched plan; trials per second from the first sweep to the boundary where the last problem
    ends."""
    def to_end(plan, chunk, label):
        plan.stream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_log = t0
        n = 0
        while True:
            plan.run(chunk)
            n += chunk
            q = plan.query()
            if q["done"].all():
                break
            if time.perf_counter() - t_log > 30:
                t_log = time.perf_counter()
                log(f"[full-run] {label}: {n} intervals, lowest stage {int(q['stage'].min())}, "
                    f"{int(q['done'].sum())} of {len(q['done'])} problems done")
        return time.perf_counter() - t0, n, q
    cfg, text = FULL_RUN[which]
    out = {"workload": text}
    one = problems(1, R, cfg)
    pp = R.Plan(one, R.Tuning(form=R.FORM_PLAIN))
    pp.init()
    Tp, _, qp = to_end(pp, 16, "plain")
    pb = R.Plan(one, R.Tuning(graph_intervals=16))
    pb.init()
    Tb, _, qb = to_end(pb, 16, "batched")
    same = all(bool((pp.walker(0, w, a)["lng"] == pb.walker(0, w, a)["lng"]).all())
               for w in range(cfg["n_windows"]) for a in range(cfg["walkers_per_window"]))
    n1 = cfg["n_windows"] * cfg["walkers_per_window"]
    trials1 = int(qp["trials"][0]) * n1
    out.update({"one_problem_trials": trials1, "plain_s": Tp, "batched_s": Tb, "plain_value": trials1 / Tp,
                "batched_value": trials1 / Tb, "speedup": Tp / Tb, "identical_final_state": same,
                "final_stage": int(qp["stage"][0])})
    pp.close()
    pb.close()
    del pp, pb
    plan = R.Plan(problems(replicas, R, cfg), R.Tuning(graph_intervals=16))
    plan.init()
    T, n, q = to_end(plan, 256, f"{replicas} replicas")
    total = int(q["trials"].sum()) * n1
    out.update({"replicas": replicas, "batch_s": T, "batch_intervals": n, "batch_trials": total,
                "batch_value": total / T, "unit": "spin-flip attempts/s",
                "trials_per_problem_min_max": [int(q["trials"].min()), int(q["trials"].max())]})
    return out


# Algorithmic VALU issue slots per trial (full-rate 32-bit lane operations; a
# 32x32->64 multiply counts 4): derivation in the design notes.
VALU_SLOTS_PER_TRIAL = 133
# MI355X: 256 CUs x 64 lanes x 2.4 GHz full-rate VALU lane operations per second.
VALU_PEAK_SLOTS = 256 * 64 * 2.4e9
# HBM-side bytes per sweep launch, FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (scales from a 1 GiB
# device copy), by (workload, replicas, table layout, walkers per workgroup, grid waves per CU,
# walkers per wavefront); measured on the current sweep kernel with rocprofv3 --pmc.  Other
# shapes report null.
TRAFFIC_BYTES = {("c4", 256, 3, 256, 4, 0): 137.60e9}
# Share of the chip's VALU cycles the sweep keeps busy by the counters (4 x SQ_ACTIVE_INST_VALU
# over 1024 SIMDs x GRBM_GUI_ACTIVE cycles per XCD), same keys; null where not measured.
VALU_BUSY = {("c4", 256, 3, 256, 4, 0): 0.370}


def launch_key(workload, replicas, layout, n_walk, wg, gw, wpw, n_cu=256):
    """Key of the measured tables above for this launch.  Shapes that differ only in `gw` are the
    same launch when both persistent grids give every tile of walkers its own workgroup (the cap
    does not bind): such a shape shares the entry measured for the other.  None when the
    walkers per workgroup are left to the library (no measured entry is claimed then)."""
    if wg <= 0:
        return None
    per = (wg // 64) * (wpw or 64)
    tiles = -(-n_walk // per)

    def grid(g):
        return tiles if g <= 0 else min(tiles, max(1, g * n_cu * 64 // wg))

    for k in TRAFFIC_BYTES:
        if k[:4] == (workload, replicas, layout, wg) and k[5] == wpw and grid(k[4]) == grid(gw):
            return k
    return (workload, replicas, layout, wg, gw, wpw)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def problems(R, R_mod, cfg=C2):
    """R replicas; cfg is one problem or a list of problems making up one replica (seed = running index)."""
    cfgs = cfg if isinstance(cfg, list) else [cfg]
    return [R_mod.Problem(seed=r * len(cfgs) + j, **c) for r in range(R) for j, c in enumerate(cfgs)]


def time_plan(R, plan, steps, warmup):
    import torch
    plan.run(warmup)
    plan.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(steps)
    plan.stream.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bench_lnz(R, torch, np):
    """ln Z forward and first-order backward (moments + grad ln g) on the 32x32 joint table shaped
    as the exact marginal g(E) (stored in tests/golden) times the binomial in M, over the grid
    beta in [0.1, 1] (1024 points) x h in [-0.5, 0.5] (256 points)."""
    import math
    N = 1024
    with open(os.path.join(ROOT, "tests", "golden", "exact_lngE.json")) as f:
        lge = np.array([-math.inf if v is None else v for v in json.load(f)["lattices"]["32"]["lnge"]])
    lbin = np.array([math.lgamma(N + 1) - math.lgamma(k + 1) - math.lgamma(N - k + 1) for k in range(N + 1)])
    lng = lge[:, None] + lbin[None, :] - N * math.log(2.0)
    b = np.linspace(0.1, 1.0, 1024)
    h = np.linspace(-0.5, 0.5, 256)
    B, Hh = np.meshgrid(b, h, indexing="ij")
    dl = torch.tensor(lng, device="cuda")
    db = torch.tensor(B.ravel(), device="cuda")
    dh = torch.tensor(Hh.ravel(), device="cuda")
    go = torch.ones_like(db)
    terms = db.numel() * int(np.isfinite(lng).sum())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    R.lnz_forward(dl, db, dh, N)                       # warm-up
    torch.cuda.synchronize()
    ev[0].record()
    z = R.lnz_forward(dl, db, dh, N)
    ev[1].record()
    gb, gh, gl = R._lnz_grads(dl, db, dh, z, go, N, 0, 0, True)
    ev[2].record()
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1])
    bwd = ev[1].elapsed_time(ev[2])
    # the same grid as a tensor product (factorised through the M columns)
    dbv, dhv = torch.tensor(b, device="cuda"), torch.tensor(h, device="cuda")
    gov = torch.ones((b.size, h.size), dtype=torch.float64, device="cuda")
    R.lnz_grid_forward(dl, dbv, dhv, N)                # warm-up
    torch.cuda.synchronize()
    ev[0].record()
    zg = R.lnz_grid_forward(dl, dbv, dhv, N)
    ev[1].record()
    R.lnz_grid_backward(dl, dbv, dhv, zg, gov, N, want_lng=True)
    ev[2].record()
    torch.cuda.synchronize()
    gfwd = ev[0].elapsed_time(ev[1])
    gbwd = ev[1].elapsed_time(ev[2])
    agree = float((zg.reshape(-1) - z).abs().max())
    return {"table": "1025 x 1025 bins (synthetic 32x32-shaped)", "grid": int(db.numel()),
            "finite_bins": int(np.isfinite(lng).sum()), "forward_ms": fwd, "backward_ms": bwd,
            "forward_terms_per_s": terms / (fwd * 1e-3),
            "backward_terms_per_s": terms / (bwd * 1e-3),
            "grid_forward_ms": gfwd, "grid_backward_ms": gbwd,
            "grid_forward_terms_per_s": terms / (gfwd * 1e-3),
            "grid_vs_direct_max_abs_diff": agree, "dtype": "f64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--replicas", type=int, default=0,
                    help="independent replicas of the workload's problem set (0 = its default, or as many as fit)")
    ap.add_argument("--layout", type=int, default=-1, help="table layout: 0 dense, 1 band, 2 dense packed, 3 band packed, -1 = choose by timing")
    ap.add_argument("--no-extras", action="store_true", help="skip the 16x16 and mixed-L workloads")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-intervals", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-lnz", action="store_true")
    ap.add_argument("--wg", type=int, default=0, help="walkers per workgroup (0 = library's choice)")
    ap.add_argument("--grid-waves", type=int, default=0, help="persistent grid waves per CU (0 = library's choice)")
    ap.add_argument("--full-run", type=int, default=0, metavar="R",
                    help="only run one problem to its end: plain, batched, and R replicas batched")
    ap.add_argument("--full-run-problem", default="c1", choices=sorted(FULL_RUN),
                    help="c1: the 4x4 serial problem; p8: the 8x8 REWL problem (3 x 3 walkers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent replicas or window blocks would shard across GPUs, but no multi-GPU path is "
              "implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1508_02748_amd as R

    if args.full_run:
        print(json.dumps(full_run(R, torch, args.full_run, args.full_run_problem)), flush=True)
        return

    dev = "cuda:0"
    K, W = args.steps, args.warmup
    unit, default_r, wl_text = WORKLOADS[args.workload]
    cfg = unit[0]
    X = cfg["interval"]
    n1 = cfg["n_windows"] * cfg["walkers_per_window"]
    from paper_1508_02748_amd.tune import autotune, choose_layout

    # ---------------- table layout and replica count
    free, total = torch.cuda.mem_get_info(0)
    budget = free - MEM_SPARE
    # replicas beyond one wavefront of walkers per SIMD would put a second wavefront on some
    # SIMDs, which then take twice as long
    walkers_per_rep = sum(c["n_windows"] * c["walkers_per_window"] for c in unit)
    one_wave_per_simd = max(1, 4 * torch.cuda.get_device_properties(0).multi_processor_count * 64 // walkers_per_rep)
    layout_report = None
    fit = None
    if args.layout >= 0:
        layout = args.layout
    else:
        layout, fit, layout_report = choose_layout(lambda r: problems(r, R, unit), budget=budget, device=dev,
                                                   max_replicas=one_wave_per_simd)
    per_rep = R.plan_bytes(problems(1, R, unit), layout)
    if args.replicas <= 0:
        args.replicas = default_r if default_r > 0 else (fit or max(1, min(one_wave_per_simd, budget // per_rep)))
    log(f"[bench] {args.workload}: layout {layout}, {per_rep / 2**30:.3f} GiB per replica, "
        f"{args.replicas} replicas ({free / 2**30:.0f} GiB free)")

    # ---------------- batched form on the replica batch (the headline value)
    tuning = R.Tuning(graph_intervals=K, walkers_per_wg=args.wg, grid_waves_per_cu=args.grid_waves,
                      table_layout=layout)
    plan = R.Plan(problems(args.replicas, R, unit), tuning, device=dev)
    t0 = time.perf_counter()
    plan.init()
    log(f"[bench] init + window entry {time.perf_counter() - t0:.2f}s; warmup {W}, timed {K} steps")
    tuned = "fixed"
    tune_report = None
    shape = (args.wg, args.grid_waves, 0)
    if not args.no_autotune and args.wg == 0 and args.grid_waves == 0:
        best = autotune(plan, intervals=1, use_cache=False)
        tune_report = plan.tune_report
        shape = (best.walkers_per_wg, best.grid_waves_per_cu, best.walkers_per_wave)
        tuned = (f"autotuned: walkers_per_wg={best.walkers_per_wg}, grid_waves_per_cu={best.grid_waves_per_cu}, "
                 f"walkers_per_wave={best.walkers_per_wave or 64}, graph_intervals={best.graph_intervals}")
        log(f"[bench] {tuned}")
    key = launch_key(args.workload, args.replicas, layout, plan.n_walkers, *shape)
    traffic = TRAFFIC_BYTES.get(key)
    valu_busy = VALU_BUSY.get(key)
    q0 = plan.query()
    # timed region: the batched launch sequence enqueued eagerly with a HIP
    # event pair around every sweep kernel on the plan's stream, so that the
    # throughput and the kernel's own duration (roofline) cover the same K
    # intervals.  The sweep gets faster over the first tens of intervals as
    # the tables fill, so both must come from the same intervals.
    plan.set_profile(True)
    T = time_plan(args.replicas, plan, K, W)
    sweep_ms = plan.sweep_times()
    # the next K intervals replayed from the captured interval graph (the
    # library's default path for rewl_run), after one untimed replay that
    # captures the graph if the autotuner's final setting dropped it
    plan.set_profile(False)
    Tg = time_plan(args.replicas, plan, K, K)
    q1 = plan.query()
    n_walk = plan.n_walkers
    active = int((~q1["done"]).sum())
    assert active == args.replicas * len(unit), "a replica finished during the timed region"
    trials = n_walk * X * K
    value = trials / T
    assert len(sweep_ms) == K
    sweep_avg = float(np.mean(sweep_ms))
    achieved_slots = VALU_SLOTS_PER_TRIAL * n_walk * X / (sweep_avg * 1e-3)
    wpw = shape[2] or 64
    waves = -(-n_walk // wpw)
    log(f"[bench] batched {value:.4e} trials/s, {T / K * 1e3:.2f} ms/step, sweep kernel {sweep_avg:.3f} ms, "
        f"{waves} wavefronts")
    stages = (int(q1["stage"].min()), int(q1["stage"].max()))
    plan.close()
    del plan
    torch.cuda.empty_cache()

    # ---------------- plain vs batched on the single problem (same trials, same final ln f)
    plain = None
    if not args.no_plain:
        Kp = args.plain_steps
        log(f"[bench] plain vs batched on one problem, {Kp} intervals each")
        pp = R.Plan(problems(1, R, cfg), R.Tuning(form=R.FORM_PLAIN, table_layout=layout), device=dev)
        pp.init()
        Tp = time_plan(1, pp, Kp, 1)
        pb = R.Plan(problems(1, R, cfg), R.Tuning(graph_intervals=Kp, table_layout=layout), device=dev)
        pb.init()
        Tb = time_plan(1, pb, Kp, 1)
        same = all((pp.walker(0, w, a)["lng"] == pb.walker(0, w, a)["lng"]).all()
                   for w in range(cfg["n_windows"]) for a in range(cfg["walkers_per_window"]))
        plain = {"workload": f"one {cfg['L']}x{cfg['L']} REWL problem ({n1} walkers)", "intervals": Kp,
                 "plain_value": n1 * X * Kp / Tp, "batched_value": n1 * X * Kp / Tb,
                 "speedup": Tp / Tb, "identical_final_state": bool(same),
                 "batched_replicas_speedup_vs_plain": value / (n1 * X * Kp / Tp)}
        log(f"[bench] plain {plain['plain_value']:.3e}, batched(1) {plain['batched_value']:.3e} trials/s")
        pp.close()
        pb.close()
        del pp, pb

    # ---------------- the other measured configurations, next to the headline
    extras = {}
    for name in ([] if args.no_extras else [n for n in ("c2", "c3mix") if n != args.workload]):
        eunit, er, etext = WORKLOADS[name]
        lay = EXTRA_LAYOUT[name]
        ep = R.Plan(problems(er, R, eunit), R.Tuning(graph_intervals=K, table_layout=lay), device=dev)
        ep.init()
        eb = autotune(ep, intervals=1, use_cache=False, graph_lengths=(K,))
        wg, gw, wpw_e = eb.walkers_per_wg, eb.grid_waves_per_cu, eb.walkers_per_wave
        ep.set_profile(True)
        eX = eunit[0]["interval"]
        Te = time_plan(er, ep, args.extra_steps, 3)
        ems = float(np.mean(ep.sweep_times()))
        ew = ep.n_walkers
        eq = ep.query()
        extras[name] = {"workload": f"{etext} x {er} independent replicas, batched form",
                        "value": ew * eX * args.extra_steps / Te, "unit": "spin-flip attempts/s",
                        "walkers": ew, "steps": args.extra_steps, "sweep_ms": ems,
                        "frac_model": VALU_SLOTS_PER_TRIAL * ew * eX / (ems * 1e-3) / VALU_PEAK_SLOTS,
                        "tuning": {"table_layout": lay, "walkers_per_wg": wg, "grid_waves_per_cu": gw,
                                   "walkers_per_wave": wpw_e or 64},
                        "stage_range": [int(eq["stage"].min()), int(eq["stage"].max())]}
        log(f"[bench] {name}: {extras[name]['value']:.3e} trials/s, sweep {ems:.2f} ms")
        ep.close()
        del ep
        torch.cuda.empty_cache()

    # ---------------- reweighting ln Z(beta, h) and its backward on the 32x32 size
    lnz = None
    if not args.no_lnz:
        lnz = bench_lnz(R, torch, np)
        log(f"[bench] lnZ forward {lnz['forward_ms']:.1f} ms, backward {lnz['backward_ms']:.1f} ms; "
            f"tensor-product grid forward {lnz['grid_forward_ms']:.2f} ms, backward {lnz['grid_backward_ms']:.2f} ms")

    # ---------------- CPU oracle on the host cores (bounded sample)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, n1, X, args.cpu_intervals)

    out = {
        "metric": METRIC, "value": value, "unit": "spin-flip attempts/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": T / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"{wl_text} x {args.replicas} independent replicas, batched form",
                   "tuning": tuned, "table_layout": ["dense", "band", "dense_packed", "band_packed"][layout],
                   "layout_probe": layout_report, "autotune": tune_report,
                   "replicas": args.replicas, "walkers": n_walk, "wavefronts": waves,
                   "bytes_per_replica": per_rep, "trials_per_walker_per_step": X,
                   "stage_range": list(stages), "stage_range_before_timing": [int(q0["stage"].min()),
                                                                             int(q0["stage"].max())],
                   "parallelism": "one walker per lane",
                   "timed": "K intervals launched eagerly, a HIP event pair around each sweep kernel",
                   "graph_replay_value": trials / Tg,
                   "graph_replay_note": "the next K intervals after an untimed K-interval replay"},
        "roofline": {"bound": "alu", "achieved": achieved_slots / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s (full-rate VALU lane-ops)", "frac": achieved_slots / VALU_PEAK_SLOTS,
                     "frac_source": f"instruction model: {VALU_SLOTS_PER_TRIAL} full-rate VALU slots per trial "
                                    "(algorithmic, counted in the design notes) x trials / sweep kernel time",
                     "valu_busy_counters": valu_busy,
                     "traffic": traffic, "traffic_unit": "HBM bytes per sweep launch (rocprofv3 FETCH_SIZE, WRITE_SIZE)",
                     "kernel": "k_sweep", "kernel_ms": sweep_avg,
                     "kernel_ms_source": "HIP events around each sweep launch of the timed intervals",
                     "slots_per_trial": VALU_SLOTS_PER_TRIAL},
        "cpu_baseline": cpu,
        "plain": plain,
        "extras": extras,
        "lnz": lnz,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, n1, X, intervals):
    """The oracle on the host: `intervals` whole intervals of one problem on all host threads, and
    a part-interval sweep on one thread (the same walkers, fresh from init)."""
    import subprocess
    from oracle.rewl import OracleREWL, set_threads
    threads = set_threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        model = next(ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name"))
    except (OSError, StopIteration, subprocess.SubprocessError):
        pass
    o = OracleREWL(seed=0, **cfg)
    o.init()
    log(f"[bench] oracle: {intervals} intervals of one {cfg['L']}x{cfg['L']} REWL problem on {threads} threads")
    Ts = Tb = 0.0
    T_first = None
    for _ in range(intervals):          # what or_run does, with the two parts timed apart
        t0 = time.perf_counter()
        o.sweep(X)
        t1 = time.perf_counter()
        o.boundary()
        Ts += t1 - t0
        Tb += time.perf_counter() - t1
        T_first = t1 - t0 if T_first is None else T_first
    Tc = Ts + Tb
    del o
    # one core: the first interval's sweep again, on one thread
    set_threads(1)
    o = OracleREWL(seed=0, **cfg)
    o.init()
    t0 = time.perf_counter()
    o.sweep(X)
    T1 = time.perf_counter() - t0
    del o
    set_threads(threads)
    return {"value": n1 * X * intervals / Tc, "unit": "spin-flip attempts/s", "cores": min(threads, n1),
            "kind": "oracle", "sweep_only_value": n1 * X * intervals / Ts,
            "first_interval_sweep_value": n1 * X / T_first, "one_core_value": n1 * X / T1,
            "host_cpu": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "sample": f"all cores: {intervals} whole intervals ({X} trials x {n1} walkers, then the boundary: a serial "
                      f"full-table flatness scan and the exchange) of one {cfg['L']}x{cfg['L']} REWL problem, seed 0, "
                      f"{Tc:.1f} s ({Ts:.1f} s in the parallel sweeps, the first one {T_first:.1f} s); one core: the "
                      f"first interval's sweep of the same problem again, {T1:.1f} s"}


if __name__ == "__main__":
    main()
