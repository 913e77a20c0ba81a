"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Spins, E, M, ln g (int64 fixed point), H, trial counts, stages and the done
flag must be identical, walker by walker, under the same Philox stream: the
acceptance is the same fixed sequence of IEEE operations on both sides, so
there is no tolerance.
"""
import sys

import numpy as np
import pytest

from oracle.rewl import OracleREWL

pytestmark = pytest.mark.gpu


def _R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_02748_amd as R
    R.lib()
    return R


def _oracle_of(p):
    mw = (p.m_windows, p.m_overlap) if p.split == 2 else None
    o = OracleREWL(p.L, p.n_windows, p.overlap, p.walkers_per_window, p.k_final, p.flat, p.interval,
                   p.seed, p.init, sync=p.stage_sync, split=p.split, m_windows=mw)
    o.init()
    return o


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(plan, pi, orc, tables=True, walkers=None):
    p = plan.problems[pi]
    gs = range(orc.n_walkers) if walkers is None else walkers
    for g in gs:
        w, a = divmod(g, p.walkers_per_window)
        dg = plan.walker(pi, w, a, tables=tables)
        do = orc.walker(g, tables=tables)
        assert (dg["e"], dg["m"], dg["t"]) == (do["e"], do["m"], do["t"]), (pi, g)
        assert (dg["spins"] == do["spins"]).all(), (pi, g)
        if tables:
            assert (dg["lng"] == do["lng"]).all(), (pi, g, "lng")
            assert (dg["H"] == do["H"].astype(np.uint64)).all(), (pi, g, "H")
    q = plan.query()
    info = orc.info()
    assert int(q["stage"][pi]) == info["stage"] and bool(q["done"][pi]) == info["done"], (q, info)
    qw = plan.query_windows(pi)
    assert plan.windows_of[pi] == orc.n_windows
    for w in range(orc.n_windows):
        assert (int(qw["stage"][w]), bool(qw["done"][w])) == orc.window_state(w), (pi, w)


def test_c1_serial_wl_full_run_bit_exact():
    R = _R()
    p = R.Problem(L=4, n_windows=1, walkers_per_window=1, k_final=16, interval=10_000, seed=0)
    _say("case: C1 4x4 serial 2D-WL, K=16, full run")
    plan = R.Plan([p])
    plan.init()
    orc = _oracle_of(p)
    compare(plan, 0, orc)
    for _ in range(100):
        plan.run(16)
        orc.run(16)
        compare(plan, 0, orc)
        if orc.info()["done"]:
            break
    assert orc.info()["done"] and bool(plan.query()["done"][0])
    # finished problems stop changing
    plan.run(5)
    compare(plan, 0, orc)


def test_c2_rewl_16x16_prefix_bit_exact():
    R = _R()
    p = R.Problem(L=16, n_windows=8, walkers_per_window=4, k_final=20, interval=10_000, seed=0)
    _say("case: C2 16x16 REWL 8x4, 48 intervals, batched graph G=8")
    plan = R.Plan([p], R.Tuning(graph_intervals=8))
    plan.init()
    orc = _oracle_of(p)
    compare(plan, 0, orc)
    for _ in range(3):
        plan.run(16)
        orc.run(16)
        compare(plan, 0, orc)


def test_plain_form_equals_batched_and_oracle():
    R = _R()
    p = R.Problem(L=8, n_windows=3, walkers_per_window=2, k_final=8, interval=1000, seed=5)
    _say("case: plain vs batched, 8x8 3x2, K=8")
    plain = R.Plan([p], R.Tuning(form=R.FORM_PLAIN))
    batched = R.Plan([p], R.Tuning(graph_intervals=4))
    plain.init()
    batched.init()
    orc = _oracle_of(p)
    for _ in range(6):
        plain.run(40)
        batched.run(40)
        orc.run(40)
        compare(plain, 0, orc)
        compare(batched, 0, orc)


def test_mixed_lattice_batch_one_launch():
    R = _R()
    probs = [R.Problem(L=8, n_windows=2, walkers_per_window=3, k_final=12, interval=2000, seed=11),
             R.Problem(L=12, n_windows=4, walkers_per_window=2, k_final=12, interval=2000, seed=12),
             R.Problem(L=16, n_windows=8, walkers_per_window=1, k_final=12, interval=2000, seed=13),
             R.Problem(L=24, n_windows=5, walkers_per_window=2, k_final=12, interval=2000, seed=14, init=1),
             R.Problem(L=32, n_windows=3, walkers_per_window=2, k_final=12, interval=2000, seed=15)]
    _say("case: mixed batch L in {8,12,16,24,32}, uneven windows")
    plan = R.Plan(probs, R.Tuning(graph_intervals=3))
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for i, o in enumerate(orcs):
        compare(plan, i, o)
    plan.run(7)
    for i, o in enumerate(orcs):
        o.run(7)
        compare(plan, i, o)


@pytest.mark.parametrize("wg,G", [(64, 1), (128, 5), (256, 2)])
def test_tuning_does_not_change_results(wg, G):
    R = _R()
    probs = [R.Problem(L=8, n_windows=3, walkers_per_window=5, k_final=10, interval=700, seed=s)
             for s in range(7)]
    _say(f"case: tuning wg={wg} G={G}")
    plan = R.Plan(probs, R.Tuning(walkers_per_wg=wg, graph_intervals=G))
    plan.init()
    plan.run(25)
    for i, p in enumerate(probs):
        o = _oracle_of(p)
        o.run(25)
        compare(plan, i, o)


def test_odd_interval_split_calls_and_boundaries():
    R = _R()
    p = R.Problem(L=6, n_windows=2, overlap=(1, 2), walkers_per_window=3, k_final=6, interval=333, seed=77)
    _say("case: odd trial counts, split sweep/reduce/exchange calls")
    plan = R.Plan([p])
    plan.init()
    orc = _oracle_of(p)
    for n in (1, 2, 3, 333, 1000, 7):
        plan.sweep(n)
        orc.sweep(n)
        compare(plan, 0, orc)
        plan.reduce_lnf()
        plan.exchange()
        orc.boundary()
        compare(plan, 0, orc)
    plan.sweep(0)
    compare(plan, 0, orc)


def test_l64_rows_of_two_words():
    R = _R()
    p = R.Problem(L=64, n_windows=4, walkers_per_window=2, k_final=20, interval=4000, seed=3)
    _say("case: 64x64, 4 windows x 2, 3 intervals")
    plan = R.Plan([p])
    plan.init()
    orc = _oracle_of(p)
    compare(plan, 0, orc, tables=False)
    plan.run(3)
    orc.run(3)
    compare(plan, 0, orc)


def test_init_all_up_entry_walks():
    R = _R()
    p = R.Problem(L=12, n_windows=6, walkers_per_window=2, k_final=10, interval=500, seed=21, init=1)
    _say("case: all-up start, entry walk into 6 windows")
    plan = R.Plan([p])
    plan.init()
    orc = _oracle_of(p)
    compare(plan, 0, orc)
    plan.run(4)
    orc.run(4)
    compare(plan, 0, orc)


def test_persistent_grid_loops_over_tiles():
    R = _R()
    # 600 problems x 32 walkers = 19,200 walkers = 300 tiles of 64 lanes, on a
    # grid of 256 workgroups (1 wavefront per CU): workgroups run several tiles
    probs = [R.Problem(L=4, n_windows=2, overlap=(1, 2), walkers_per_window=16, k_final=8, interval=300, seed=s)
             for s in range(600)]
    _say("case: persistent grid, 300 tiles on 256 workgroups")
    plan = R.Plan(probs, R.Tuning(walkers_per_wg=64, grid_waves_per_cu=1, graph_intervals=2))
    plan.init()
    plan.run(6)
    for i in (0, 1, 299, 598, 599):
        o = _oracle_of(probs[i])
        o.run(6)
        compare(plan, i, o)


def test_per_window_variant_bit_exact_batched_and_plain():
    """REWL_SYNC_WINDOW: windows refine alone after averaging their walkers; run
    past the point where some windows have finished and others have not."""
    R = _R()
    p = R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=3, k_final=5, interval=1000, seed=3,
                  stage_sync=R.SYNC_WINDOW)
    _say("case: per-window variant 8x8 3x3, K=5, batched and plain (the oracle ends after 3680 intervals)")
    batched = R.Plan([p], R.Tuning(graph_intervals=4))
    plain = R.Plan([p], R.Tuning(form=R.FORM_PLAIN))
    batched.init()
    plain.init()
    orc = _oracle_of(p)
    seen_partial = False
    for _ in range(300):
        batched.run(20)
        plain.run(20)
        orc.run(20)
        compare(batched, 0, orc)
        compare(plain, 0, orc)
        ws = [orc.window_state(w)[1] for w in range(p.n_windows)]
        seen_partial = seen_partial or (any(ws) and not all(ws))
        if orc.info()["done"]:
            break
    assert orc.info()["done"] and seen_partial


def test_mixed_sync_batch_bit_exact():
    """Problems of both stage rules and several lattice sizes in one launch."""
    R = _R()
    probs = [R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=21,
                       stage_sync=R.SYNC_WINDOW),
             R.Problem(L=12, n_windows=4, walkers_per_window=2, k_final=8, interval=1000, seed=22),
             R.Problem(L=16, n_windows=4, walkers_per_window=3, k_final=8, interval=1000, seed=23,
                       stage_sync=R.SYNC_WINDOW),
             R.Problem(L=4, n_windows=1, walkers_per_window=4, k_final=10, interval=1000, seed=24,
                       stage_sync=R.SYNC_WINDOW)]
    _say("case: mixed stage rules, L in {4,8,12,16}")
    plan = R.Plan(probs, R.Tuning(graph_intervals=5))
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for _ in range(12):
        plan.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(plan, i, o)


def test_degenerate_sizes_bit_exact():
    """k_final = 0 (one stage), an interval of one trial (every sweep starts or
    ends in the middle of a Philox block), and 256 walkers per window."""
    R = _R()
    cases = [
        ("K=0, X=7", R.Problem(L=4, n_windows=1, walkers_per_window=1, k_final=0, interval=7, seed=9), 5, 1),
        ("X=1, per-window rule", R.Problem(L=6, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=3,
                                            interval=1, seed=4, stage_sync=R.SYNC_WINDOW), 3000, 500),
        ("X=1, problem rule",
         R.Problem(L=8, n_windows=2, walkers_per_window=3, k_final=4, interval=1, seed=6), 2000, 400),
        ("256 walkers per window", R.Problem(L=4, n_windows=2, overlap=(1, 2), walkers_per_window=256, k_final=4,
                                             interval=50, seed=5), 100, 25),
    ]
    for name, p, total, step in cases:
        _say("case:", name)
        plan = R.Plan([p], R.Tuning(graph_intervals=4))
        plan.init()
        orc = _oracle_of(p)
        done = 0
        while done < total:
            plan.run(step)
            orc.run(step)
            done += step
            compare(plan, 0, orc)


def test_walkers_per_wave_shapes_bit_exact():
    """Fewer walkers per wavefront (a small batch spread over more CUs) and any
    workgroup size give the same trajectories."""
    R = _R()
    probs = [R.Problem(L=8, n_windows=3, walkers_per_window=5, k_final=8, interval=700, seed=40),
             R.Problem(L=12, n_windows=2, walkers_per_window=7, k_final=8, interval=700, seed=41)]
    orcs = [_oracle_of(p) for p in probs]
    for o in orcs:
        o.run(12)
    for wg, wpw in ((64, 1), (64, 5), (128, 37), (256, 3), (256, 64)):
        _say("case: walkers_per_wg", wg, "walkers_per_wave", wpw)
        for form in (R.FORM_BATCHED, R.FORM_PLAIN):
            plan = R.Plan(probs, R.Tuning(form=form, walkers_per_wg=wg, walkers_per_wave=wpw,
                                          graph_intervals=3 if form == R.FORM_BATCHED else 0))
            plan.init()
            plan.run(12)
            for i, o in enumerate(orcs):
                compare(plan, i, o)
