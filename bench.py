"""Throughput of two-dimensional replica-exchange Wang-Landau sampling on one MI355X.

One step = one REWL interval over the whole batch: 10^4 Wang-Landau trials per
walker (Eq. 1 random walk in (E, M)), the flatness check and ln f reduction,
and one exchange round between adjacent windows (Eq. 2).

Workload: the 16x16 periodic Ising REWL problem (8 energy windows with 3/4
overlap, full M range, 4 walkers per window, ln f from 1 to 2^-20, 80 %
flatness, exchange every 10^4 trials, random initial spins) replicated with
independent seeds so that one walker per lane fills the GPU.  Inputs are
synthetic (seeded spins); every table and configuration is resident in HBM
before the timed region.

Prints one JSON line: batched throughput (value), the plain
one-launch-per-window form on the single problem next to the batched form on
the same problem (same trials, so the same final ln f), the roofline of the
sweep kernel (timed with HIP events around each of its launches) and the
CPU oracle on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/sec on 1 MI355X (batched vs plain) at equal final ln f"
# One 16x16 REWL problem: the configuration the throughput is quoted on.
C2 = dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=20, flat=(4, 5), interval=10_000)
# Algorithmic VALU issue slots per trial (full-rate 32-bit lane operations; a
# 32x32->64 multiply counts 4): derivation in the design notes.
VALU_SLOTS_PER_TRIAL = 133
# MI355X: 256 CUs x 64 lanes x 2.4 GHz full-rate VALU lane operations per second.
VALU_PEAK_SLOTS = 256 * 64 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def problems(R, R_mod):
    return [R_mod.Problem(seed=s, **C2) for s in range(R)]


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replicas", type=int, default=4096)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--cpu-intervals", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--wg", type=int, default=0, help="walkers per workgroup (0 = library's choice)")
    ap.add_argument("--grid-waves", type=int, default=0, help="persistent grid waves per CU (0 = library's choice)")
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
              "independent replicas or window blocks would shard across GPUs, but this build has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1508_02748_amd as R

    dev = "cuda:0"
    K, W = args.steps, args.warmup
    X = C2["interval"]

    # ---------------- batched form on the replica batch (the headline value)
    log(f"[bench] batched: {args.replicas} replicas of the 16x16 REWL problem, init ...")
    tuning = R.Tuning(graph_intervals=K, walkers_per_wg=args.wg, grid_waves_per_cu=args.grid_waves)
    plan = R.Plan(problems(args.replicas, R), tuning, device=dev)
    t0 = time.perf_counter()
    plan.init()
    log(f"[bench] init + window entry {time.perf_counter() - t0:.2f}s; warmup {W}, timed {K} steps")
    # timed region: the batched launch sequence enqueued eagerly with a HIP
    # event pair around every sweep kernel on the plan's stream
    plan.set_profile(True)
    T = time_plan(args.replicas, plan, K, W)
    sweep_ms = plan.sweep_times()
    # the same K intervals replayed from the captured interval graph
    plan.set_profile(False)
    Tg = time_plan(args.replicas, plan, K, 0)
    q1 = plan.query()
    n_walk = plan.n_walkers
    active = int((~q1["done"]).sum())
    assert active == args.replicas, "a replica finished during the timed region"
    trials = n_walk * X * K
    value = trials / T
    assert len(sweep_ms) == K
    sweep_avg = float(np.mean(sweep_ms))
    achieved_slots = VALU_SLOTS_PER_TRIAL * n_walk * X / (sweep_avg * 1e-3)
    log(f"[bench] batched {value:.4e} trials/s, {T / K * 1e3:.2f} ms/step, sweep kernel {sweep_avg:.3f} ms")
    stages = (int(q1["stage"].min()), int(q1["stage"].max()))
    del plan
    torch.cuda.empty_cache()

    # ---------------- plain vs batched on the single problem (same trials, same final ln f)
    plain = None
    if not args.no_plain:
        Kp = args.plain_steps
        log(f"[bench] plain vs batched on one problem, {Kp} intervals each")
        pp = R.Plan(problems(1, R), R.Tuning(form=R.FORM_PLAIN), device=dev)
        pp.init()
        Tp = time_plan(1, pp, Kp, 1)
        pb = R.Plan(problems(1, R), R.Tuning(graph_intervals=Kp), device=dev)
        pb.init()
        Tb = time_plan(1, pb, Kp, 1)
        same = all((pp.walker(0, w, a)["lng"] == pb.walker(0, w, a)["lng"]).all()
                   for w in range(C2["n_windows"]) for a in range(C2["walkers_per_window"]))
        n1 = C2["n_windows"] * C2["walkers_per_window"]
        plain = {"workload": "one 16x16 REWL problem (32 walkers)", "intervals": Kp,
                 "plain_value": n1 * X * Kp / Tp, "batched_value": n1 * X * Kp / Tb,
                 "speedup": Tp / Tb, "identical_final_state": bool(same),
                 "batched_replicas_speedup_vs_plain": value / (n1 * X * Kp / Tp)}
        log(f"[bench] plain {plain['plain_value']:.3e}, batched(1) {plain['batched_value']:.3e} trials/s")
        del pp, pb

    # ---------------- CPU oracle on the host cores (bounded sample)
    cpu = None
    if not args.no_cpu:
        from oracle.rewl import OracleREWL
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        o = OracleREWL(seed=0, **{"L": 16, "n_windows": 8, "overlap": (3, 4), "walkers_per_window": 4,
                                  "k_final": 20, "flat": (4, 5), "interval": X})
        o.init()
        n = args.cpu_intervals
        log(f"[bench] oracle: {n} intervals of one 16x16 REWL problem on {threads} threads")
        t0 = time.perf_counter()
        o.run(n)
        Tc = time.perf_counter() - t0
        cpu = {"value": 32 * X * n / Tc, "unit": "spin-flip attempts/s", "cores": min(threads, 32),
               "kind": "oracle",
               "sample": f"{n} intervals (10^4 trials x 32 walkers each) of one 16x16 REWL problem, seed 0; "
                         f"{Tc:.1f} s"}

    out = {
        "metric": METRIC, "value": value, "unit": "spin-flip attempts/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": T / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"16x16 periodic Ising 2D-REWL (8 windows x 4 walkers, overlap 3/4, "
                               f"ln f 1 -> 2^-20, 80% flat, exchange every 10^4 trials) x {args.replicas} "
                               f"independent replicas, batched form",
                   "replicas": args.replicas, "walkers": n_walk, "trials_per_walker_per_step": X,
                   "stage_range": list(stages), "parallelism": "one walker per lane",
                   "graph_replay_value": trials / Tg},
        "roofline": {"bound": "alu", "achieved": achieved_slots / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s (full-rate VALU lane-ops)", "frac": achieved_slots / VALU_PEAK_SLOTS,
                     "traffic": None, "kernel": "k_sweep", "kernel_ms": sweep_avg,
                     "slots_per_trial": VALU_SLOTS_PER_TRIAL},
        "cpu_baseline": cpu,
        "plain": plain,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
