"""Long GPU runs to convergence, compared with the exact g(E) (not a pytest file).

Runs REWL problems on the GPU until every problem has finished its last stage
(resumable across calls through rewl_save / rewl_load checkpoints), joins each
problem's fragments on the device (Eq. 3, Eq. 4) and compares the marginal
ln g(E) with the exact finite-lattice values stored in tests/golden/ (Sec. 3,
Fig. 5):  epsilon(E) = |ln g - ln g_exact| / ln g_exact over realizable E.

  python tests/long_convergence.py --config c2 --replicas 8 --seconds 900 --out runs/conv_c2
  python tests/long_convergence.py --config c2 ... --resume      # continue from the checkpoint
  python tests/long_convergence.py --config c2 ... --resume --evaluate-now   # compare the state reached

Configurations: c2 = 16x16, 8 windows (overlap 3/4) x 4 walkers, ln f -> 2^-20;
p8w2 / p8w20 = 8x8, 3 windows (overlap 1/2) x 2 or 20 walkers, ln f -> 2^-20;
p8pair = 8x8 serial 2D-WL (one walker over the whole (E, M) space) next to
8x8 2D-REWL (3 windows, overlap 1/2, 3 walkers), both to ln f = 2^-20, with
the relative difference of Eq. 5 between the two joint densities of states
(Sec. 3, Fig. 4(b)); p8sync = the same 8x8 REWL problem with all windows
refining together (the paper) and with each window refining alone after
averaging its walkers, compared in accuracy and in trials to finish.
Replica r uses seed r (the second group uses seed 1000 + r).  Progress is
printed every minute.

  python tests/long_convergence.py --config c2 --replicas 64 --seconds 780 --decompose --out runs/dec

--decompose runs for the given time and then splits the error of the joined
marginal ln g(E) at every energy, per replica, into (1) the error of the window
piece that supplies it, after the piece is shifted by the one constant that fits
it best to the exact ln g(E) over its window (the piece error, Eq. 3), and (2)
the difference between the joint's actual matching constants (E_mat, Eq. 4) and
those best-fit constants (the join error), both after the same sum
normalisation; reported as mean and standard error over the replicas at the two
edge states E = -2N, +2N and at the next levels.
"""
import argparse
import json
import math
import os
import sys
import time
import zlib

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

P8 = dict(L=8, overlap=(1, 2), k_final=20, interval=10_000)
CONFIGS = {
    "c2": [dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=20, interval=10_000)],
    "p8w2": [dict(P8, n_windows=3, walkers_per_window=2)],
    "p8w20": [dict(P8, n_windows=3, walkers_per_window=20)],
    "p8pair": [dict(P8, n_windows=3, walkers_per_window=3), dict(P8, n_windows=1, walkers_per_window=1)],
    "p8sync": [dict(P8, n_windows=3, walkers_per_window=3),
               dict(P8, n_windows=3, walkers_per_window=3, stage_sync=1)],
    # 16x16 in one plan: the measured REWL problem (8 windows, overlap 3/4, 4 walkers), the paper's
    # own 16x16 shape (3 windows, overlap 1/2, 3 walkers; Sec. 3) and serial 2D-WL over the whole
    # (E, M) space (Fig. 4(b)); all three share X = 10^4, so they run side by side at no extra cost
    "c2p16": [dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=20, interval=10_000),
              dict(L=16, n_windows=3, overlap=(1, 2), walkers_per_window=3, k_final=20, interval=10_000),
              dict(L=16, n_windows=1, overlap=(1, 2), walkers_per_window=1, k_final=20, interval=10_000)],
}


def exact_lnge(L):
    with open(os.path.join(ROOT, "tests", "golden", "exact_lngE.json")) as f:
        ent = json.load(f)["lattices"][str(L)]
    return np.array([-math.inf if v is None else v for v in ent["lnge"]])


def rel_diff(a, b):
    """Eq. 5 from logarithms: |g1 - g2| / ((g1 + g2) / 2) = 2 |tanh((ln g1 - ln g2) / 2)|."""
    return 2.0 * np.abs(np.tanh(0.5 * (a - b)))


def paper_pair(R, plan, probs, tags, L):
    """Groups 1 (REWL) and 2 (serial 2D-WL) of each replica, evaluated where they are: the relative
    error of the marginal against the exact g(E) (sum normalisation), and Eq. 5 between the two
    joint DOS over the bins both visited (Sec. 3, Fig. 4(b) and Fig. 5(a))."""
    N = L * L
    ex = exact_lnge(L)
    ok = np.isfinite(ex) & (ex > 0)
    by = {}
    for i, (gi, r) in enumerate(tags):
        if gi in (1, 2):
            by.setdefault(r, {})[gi] = i
    rows = []
    for r, d in sorted(by.items()):
        out = {"replica": r}
        joints = {}
        for gi, i in d.items():
            q = plan.query_windows(i)
            j, g, em = plan.merge(i, "sum")
            g = g.cpu().numpy()
            eps = np.abs(g[ok] - ex[ok]) / ex[ok]
            joints[gi] = j.cpu().numpy()
            out[("rewl", "serial")[gi - 1]] = {
                "stage": int(q["stage"].min()), "trials_per_walker": int(q["trials"][0]),
                "max_eps": float(eps.max()), "mean_eps": float(eps.mean()),
                "max_eps_inner": float(eps[1:-1].max()), "bins_visited": int(np.isfinite(joints[gi]).sum())}
        a, b = joints[1], joints[2]
        both = np.isfinite(a) & np.isfinite(b)
        dd = rel_diff(a[both], b[both])
        e_rows = np.nonzero(both)[0]
        edge = (e_rows <= 2) | (e_rows >= N - 2)
        out["eq5"] = {"bins": int(both.sum()), "only_one": int((np.isfinite(a) ^ np.isfinite(b)).sum()),
                      "mean": float(dd.mean()), "median": float(np.median(dd)), "max": float(dd.max()),
                      "mean_interior": float(dd[~edge].mean()), "mean_edges": float(dd[edge].mean())}
        rows.append(out)
    summ = {}
    for key in ("rewl", "serial"):
        for f in ("stage", "max_eps", "mean_eps", "max_eps_inner"):
            v = np.array([row[key][f] for row in rows], dtype=float)
            summ[f"{key}.{f}"] = [float(v.min()), float(np.median(v)), float(v.max())]
    for f in ("mean", "median", "mean_interior", "mean_edges"):
        v = np.array([row["eq5"][f] for row in rows])
        summ[f"eq5.{f}"] = [float(v.min()), float(np.median(v)), float(v.max())]
    return {"summary": summ, "per_replica": rows}


def decompose(R, plan, probs, L, meta, index=None):
    """Piece and join parts of each replica's marginal error (see the module notes)."""
    from oracle import merge as MG
    N = L * L
    ex = exact_lnge(L)
    ok = np.isfinite(ex) & (ex > 0)
    lse = MG._lse
    rows = []
    index = list(range(len(probs))) if index is None else index
    for i, p in zip(index, probs):
        pieces = []
        for w in range(p.n_windows):
            frags = [plan.walker(i, w, a)["lng"] for a in range(p.walkers_per_window)]
            lo, hi = plan.window(i, w)
            pieces.append((lo, hi, MG.window_average(frags, p.k_final)))
        joint, marg, emats = MG.merge(pieces, N, "sum")
        # best-fit constant of each piece's marginal against the exact ln g(E)
        fit, resid = [], np.full(N + 1, np.nan)
        for w, (lo, hi, t) in enumerate(pieces):
            m = MG.marginal(t)
            sel = np.isfinite(m) & ok[lo:hi + 1]
            fit.append(float(np.mean(ex[lo:hi + 1][sel] - m[sel])))
        # exact-shift join: every piece moved by its best-fit constant, rows taken from the same
        # piece as in the actual join, then the same sum normalisation
        bounds = [0] + list(emats) + [N + 1]
        exact_join = np.full(N + 1, -np.inf)
        for w, (lo, hi, t) in enumerate(pieces):
            a, b = max(bounds[w], lo), min(bounds[w + 1], hi + 1)
            exact_join[a:b] = MG.marginal(t)[a - lo:b - lo] + fit[w]
            resid[a:b] = exact_join[a:b] - ex[a:b]
        fin = np.isfinite(exact_join)
        exact_join = exact_join - lse(exact_join[fin]) + N * math.log(2.0)
        piece_err = exact_join - ex          # error with exact matching constants
        total_err = marg - ex                # error of the actual joint
        join_err = total_err - piece_err     # what the E_mat joins add
        rows.append({"replica": i, "e_mat": [int(x) for x in emats],
                     "total": {int(e): float(total_err[e]) for e in (0, 2, 3, N - 3, N - 2, N)},
                     "piece": {int(e): float(piece_err[e]) for e in (0, 2, 3, N - 3, N - 2, N)},
                     "join": {int(e): float(join_err[e]) for e in (0, 2, 3, N - 3, N - 2, N)},
                     "piece_residual_edges": [float(resid[0]), float(resid[N])],
                     "max_eps": float(np.max(np.abs(total_err[ok]) / ex[ok])),
                     "max_eps_inner": float(np.max((np.abs(total_err[ok]) / ex[ok])[1:-1]))})
    summ = {}
    for part in ("total", "piece", "join"):
        for e in (0, 2, 3, N - 3, N - 2, N):
            v = np.array([r[part][e] for r in rows])
            v = v[np.isfinite(v)]
            summ[f"{part}@E={4 * e - 2 * N}"] = {"mean": float(v.mean()), "se": float(v.std(ddof=1) / np.sqrt(v.size)),
                                                "rms": float(np.sqrt((v ** 2).mean())), "n": int(v.size)}
    q = plan.query()
    st = q["stage"][index]
    tr = q["trials"][index]
    return {"replicas": len(probs), "stage_min_max": [int(st.min()), int(st.max())],
            "trials_per_walker_min_max": [int(tr.min()), int(tr.max())],
            "seconds": meta["seconds"], "summary": summ,
            "max_eps_per_replica": [r["max_eps"] for r in rows],
            "max_eps_inner_per_replica": [r["max_eps_inner"] for r in rows], "per_replica": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--replicas", type=int, default=8)
    ap.add_argument("--seconds", type=float, default=900)
    ap.add_argument("--out", default="runs/conv")
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--evaluate-now", action="store_true",
                    help="compare the current (unfinished) state with the exact g(E) instead of running on")
    ap.add_argument("--decompose", action="store_true",
                    help="after --seconds, split the marginal's error into piece and join errors (see above)")
    args = ap.parse_args()
    import torch  # noqa: F401  (device memory for the plan)
    import paper_1508_02748_amd as R

    os.makedirs(args.out, exist_ok=True)
    groups = CONFIGS[args.config]
    probs, tags = [], []
    for gi, cfg in enumerate(groups):
        for r in range(args.replicas):
            probs.append(R.Problem(seed=1000 * gi + r, **cfg))
            tags.append((gi, r))
    plan = R.Plan(probs, R.Tuning(graph_intervals=64))
    ck = os.path.join(args.out, "checkpoint.z")
    meta_path = os.path.join(args.out, "progress.json")
    meta = {"intervals": 0, "seconds": 0.0}
    if args.resume and os.path.exists(ck):
        with open(ck, "rb") as f:
            plan.load(zlib.decompress(f.read()))
        with open(meta_path) as f:
            meta = json.load(f)
        print(f"resumed at {meta['intervals']} intervals", flush=True)
    else:
        plan.init()
    t0 = time.time()
    last = t0
    while not args.evaluate_now and time.time() - t0 < args.seconds:
        plan.run(256)
        meta["intervals"] += 256
        q = plan.query()
        if q["done"].all():
            break
        if time.time() - last > 60:
            last = time.time()
            print(f"[{args.config}] {meta['intervals']} intervals, stages {int(q['stage'].min())}..{int(q['stage'].max())}, "
                  f"{int(q['done'].sum())}/{len(probs)} done, {time.time() - t0:.0f}s", flush=True)
    meta["seconds"] += time.time() - t0
    q = plan.query()
    if args.decompose:
        g0 = [i for i, (gi, _) in enumerate(tags) if gi == 0]
        res = decompose(R, plan, [probs[i] for i in g0], groups[0]["L"], meta, index=g0)
        if len(groups) == 3:
            res["paper_shape"] = paper_pair(R, plan, probs, tags, groups[0]["L"])
        with open(os.path.join(args.out, "decompose.json"), "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res["summary"]), flush=True)
        if "paper_shape" in res:
            print(json.dumps(res["paper_shape"]["summary"]), flush=True)
        return
    meta["done"] = int(q["done"].sum())
    meta["stage"] = [int(x) for x in q["stage"]]
    meta["trials_per_walker"] = [int(x) for x in q["trials"]]
    if not q["done"].all() and not args.evaluate_now:
        with open(ck, "wb") as f:
            f.write(zlib.compress(plan.save(), 6))
        with open(meta_path, "w") as f:
            json.dump(meta, f)
        print(f"checkpoint written: {meta['intervals']} intervals, {meta['done']}/{len(probs)} done", flush=True)
        return
    L = groups[0]["L"]
    ex = exact_lnge(L)
    ok = np.isfinite(ex) & (ex > 0)
    E_of = 4 * np.arange(ex.size)[ok] - 2 * L * L        # energies of the compared bins
    inner = np.abs(E_of) < 2 * L * L                     # all but the two edge states E = -2N, +2N
    res = {"config": args.config,
           "problems": [{k: list(v) if isinstance(v, tuple) else v for k, v in c.items()} for c in groups],
           "replicas": args.replicas, **meta, "per_replica": []}
    margs = {gi: [] for gi in range(len(groups))}
    joints = {}
    for i, (gi, r) in enumerate(tags):
        qw = plan.query_windows(i)
        out = {"group": gi, "replica": r, "window_trials_per_walker": [int(x) for x in qw["trials"]]}
        for norm in ("ground", "sum"):
            jt, g, em = plan.merge(i, norm)
            g = g.cpu().numpy()
            eps = np.abs(g[ok] - ex[ok]) / ex[ok]
            out[norm] = {"max_eps": float(eps.max()), "mean_eps": float(eps.mean()),
                         "max_abs": float(np.max(np.abs(g[ok] - ex[ok]))), "e_mat": em,
                         "E_of_max_eps": int(E_of[int(np.argmax(eps))]),
                         "max_eps_without_edges": float(eps[inner].max()),
                         # signed ln g - ln g_exact at the three lowest and three highest energies
                         "signed_err_ends": {int(E): float(v) for E, v in
                                             zip(np.r_[E_of[:3], E_of[-3:]], np.r_[(g[ok] - ex[ok])[:3],
                                                                                  (g[ok] - ex[ok])[-3:]])}}
            if norm == "sum":
                margs[gi].append(g)
                joints[(gi, r)] = jt.cpu().numpy()
        res["per_replica"].append(out)
        print(f"group {gi} replica {r}: max eps ground {out['ground']['max_eps']:.4g} sum {out['sum']['max_eps']:.4g}",
              flush=True)
    # mean over replicas and jackknife error of that mean (sum normalisation), per group
    res["replica_mean"] = []
    for gi in range(len(groups)):
        M = np.array(margs[gi])[:, ok]
        n = M.shape[0]
        mean = M.mean(0)
        jk = np.array([(M.sum(0) - M[k]) / (n - 1) for k in range(n)])
        err = np.sqrt((n - 1) / n * ((jk - jk.mean(0)) ** 2).sum(0))
        eps_mean = np.abs(mean - ex[ok]) / ex[ok]
        res["replica_mean"].append({"group": gi, "max_eps": float(eps_mean.max()), "mean_eps": float(eps_mean.mean()),
                                    "max_eps_without_edges": float(eps_mean[inner].max()),
                                    "max_jackknife_err": float(err.max()),
                                    "max_abs_over_err": float(np.max(np.abs(mean - ex[ok]) / np.maximum(err, 1e-300)))})
    for gi in range(len(groups)):
        tw = [sum(o["window_trials_per_walker"]) / len(o["window_trials_per_walker"])
              for o in res["per_replica"] if o["group"] == gi]
        res["replica_mean"][gi]["mean_trials_per_walker_to_finish"] = float(np.mean(tw))
    if args.config == "p8pair":
        # Eq. 5 between the REWL (group 0) and serial WL (group 1) joint DOS of each replica pair
        diffs = []
        for r in range(args.replicas):
            a, b = joints[(0, r)], joints[(1, r)]
            both = np.isfinite(a) & np.isfinite(b)
            d = rel_diff(a[both], b[both])
            e_rows = np.nonzero(both)[0]
            edge = (e_rows <= 2) | (e_rows >= L * L - 2)
            diffs.append({"replica": r, "bins": int(both.sum()),
                          "only_one": int((np.isfinite(a) ^ np.isfinite(b)).sum()),
                          "max": float(d.max()), "mean": float(d.mean()), "median": float(np.median(d)),
                          "mean_interior": float(d[~edge].mean()), "mean_edges": float(d[edge].mean())})
            print(f"replica {r}: Eq. 5 over {both.sum()} bins: mean {d.mean():.4g}, max {d.max():.4g}", flush=True)
        res["rel_diff"] = diffs
    name = "result.json" if q["done"].all() else "result_at_stage_%d.json" % min(meta["stage"])
    with open(os.path.join(args.out, name), "w") as f:
        json.dump(res, f, indent=1)
    if os.path.exists(ck) and q["done"].all():
        os.remove(ck)
    print(json.dumps(res["replica_mean"]), flush=True)


if __name__ == "__main__":
    main()
