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
