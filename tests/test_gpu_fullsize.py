"""Parity at the measured sizes, in the launch configuration bench.py times.

The batch is too large for the oracle as a whole, so whole replicas (problems)
are sampled and recomputed one by one; replicas are independent, so a sampled
replica's spins, E, M, ln g and H must equal the oracle's bit for bit."""
import pytest

from tests.test_gpu_parity import _R, _oracle_of, _say, compare

pytestmark = pytest.mark.gpu

C2 = dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=20, flat=(4, 5), interval=10_000)


def test_bench_configuration_sampled_replicas():
    R = _R()
    K, W = 20, 3
    probs = [R.Problem(seed=s, **C2) for s in range(4096)]
    _say("case: 16x16 REWL x 4096 replicas, bench launch configuration, 43 intervals")
    plan = R.Plan(probs, R.Tuning(graph_intervals=K))
    plan.init()
    plan.set_profile(True)
    plan.run(W)
    plan.run(K)
    plan.set_profile(False)
    plan.run(K)
    for i in (0, 2047, 4095):
        o = _oracle_of(probs[i])
        o.run(W + 2 * K)
        compare(plan, i, o)


def test_32x32_and_mixed_batch_sampled():
    R = _R()
    probs = [R.Problem(L=32, n_windows=16, walkers_per_window=8, k_final=24, interval=10_000, seed=100 + s)
             for s in range(32)]
    mixed = []
    for L, nw in ((8, 2), (12, 4), (16, 8), (24, 12), (32, 16)):
        mixed += [R.Problem(L=L, n_windows=nw, walkers_per_window=8, k_final=24, interval=10_000, seed=1000 * L + s)
                  for s in range(16)]
    _say("case: 32x32 16x8 x 32 + mixed L batch x 16, 3 intervals")
    plan = R.Plan(probs + mixed)
    plan.init()
    plan.run(3)
    for i in (0, 31, 32, 32 + 16 + 5, 32 + 48 + 7, len(probs) + len(mixed) - 1):
        o = _oracle_of((probs + mixed)[i])
        o.run(3)
        compare(plan, i, o)


def test_64x64_bench_configuration_sampled_replicas():
    """The 64x64 REWL problem (64 windows x 4 walkers, overlap 3/4, X = 1e5) x as many replicas as
    the device holds in the packed band layout, at most one wavefront per SIMD (256 on a 288 GB
    MI355X), with a 256-walker workgroup and a grid of 6 waves per CU, through eager, profiled
    and graph-replayed intervals.  The first, a middle and the last replica are recomputed by the
    oracle: every walker's spins, E, M and trial count, and the tables of a spread of walkers."""
    import torch
    R = _R()
    C4 = dict(L=64, n_windows=64, overlap=(3, 4), walkers_per_window=4, k_final=20, flat=(4, 5), interval=100_000)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info(0)
    per = R.plan_bytes([R.Problem(seed=0, **C4)], R.LAYOUT_BAND_PACKED)
    n = int(max(1, min(256, (free - (12 << 30)) // per)))
    _say(f"case: 64x64 REWL x {n} replicas, packed band layout, 256/6, 5 intervals")
    probs = [R.Problem(seed=s, **C4) for s in range(n)]
    plan = R.Plan(probs, R.Tuning(table_layout=R.LAYOUT_BAND_PACKED, walkers_per_wg=256, grid_waves_per_cu=6,
                                  graph_intervals=2))
    plan.init()
    plan.run(1)
    plan.set_profile(True)
    plan.run(2)
    plan.set_profile(False)
    plan.run(2)
    for i in sorted({0, n // 2, n - 1}):
        o = _oracle_of(probs[i])
        o.run(5)
        compare(plan, i, o, walkers=[0, 1, 2, 3, 100, 127, 128, 201, 252, 255])
        compare(plan, i, o, tables=False)
    plan.close()
    del plan
    torch.cuda.empty_cache()


def test_64x64_prefix_sampled_walkers():
    R = _R()
    p = R.Problem(L=64, n_windows=64, walkers_per_window=4, k_final=20, interval=100_000, seed=7)
    _say("case: 64x64 REWL 64x4, X=1e5, 2 intervals")
    plan = R.Plan([p])
    plan.init()
    plan.run(2)
    o = _oracle_of(p)
    o.run(2)
    compare(plan, 0, o, walkers=[0, 1, 127, 128, 252, 255])
    compare(plan, 0, o, tables=False)
