"""The band table layout (each energy row keeps only the magnetization band that
can hold states; magnetization windows keep only the energy rows that can)
changes memory and addressing, not results: bit-exact parity with the CPU
oracle, which stores whole rectangles, in both forms, both stage rules, both
one-coordinate splits, mixed lattice sizes and the full 64 x 64 size."""
import numpy as np
import pytest

from tests.test_gpu_parity import _R, _oracle_of, _say, compare

pytestmark = pytest.mark.gpu


def _band(R, **kw):
    return R.Tuning(table_layout=R.LAYOUT_BAND, **kw)


def test_band_16x16_prefix_batched_and_plain():
    R = _R()
    p = R.Problem(L=16, n_windows=8, walkers_per_window=4, k_final=20, interval=10_000, seed=0)
    _say("case: band layout, 16x16 REWL 8x4, 48 intervals, batched and plain")
    batched = R.Plan([p], _band(R, graph_intervals=8))
    plain = R.Plan([p], _band(R, form=R.FORM_PLAIN))
    assert sum(batched.sizes) < sum(R.Plan([p]).sizes)
    batched.init()
    plain.init()
    orc = _oracle_of(p)
    for _ in range(3):
        batched.run(16)
        plain.run(16)
        orc.run(16)
        compare(batched, 0, orc)
        compare(plain, 0, orc)


def test_band_mixed_lattices_and_stage_rules():
    R = _R()
    probs = [R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=21,
                       stage_sync=R.SYNC_WINDOW),
             R.Problem(L=12, n_windows=4, walkers_per_window=2, k_final=8, interval=1000, seed=22),
             R.Problem(L=24, n_windows=6, walkers_per_window=2, k_final=8, interval=1000, seed=23, init=1),
             R.Problem(L=32, n_windows=3, walkers_per_window=2, k_final=8, interval=1000, seed=24,
                       stage_sync=R.SYNC_WINDOW)]
    _say("case: band layout, L in {8,12,24,32}, both stage rules, 300 intervals")
    plan = R.Plan(probs, _band(R, graph_intervals=5))
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for _ in range(12):
        plan.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(plan, i, o)


def test_band_per_window_rule_to_the_end():
    R = _R()
    p = R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=3, k_final=5, interval=1000, seed=3,
                  stage_sync=R.SYNC_WINDOW)
    _say("case: band layout, per-window rule 8x8 3x3 K=5 to the end")
    plan = R.Plan([p], _band(R, graph_intervals=4))
    plan.init()
    orc = _oracle_of(p)
    for _ in range(300):
        plan.run(20)
        orc.run(20)
        if orc.info()["done"]:
            break
    assert orc.info()["done"]
    compare(plan, 0, orc)


def test_band_magnetization_split():
    R = _R()
    M = R.SPLIT_MAGNETIZATION
    # windows away from m = N/2 keep only the energy rows up to twice their largest minority count
    probs = [R.Problem(L=8, n_windows=5, overlap=(1, 2), walkers_per_window=3, k_final=8, interval=1000, seed=31,
                       split=M),
             R.Problem(L=16, n_windows=8, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=33,
                       split=M, stage_sync=R.SYNC_WINDOW)]
    _say("case: band layout, magnetization split, 150 intervals")
    plan = R.Plan(probs, _band(R, graph_intervals=5))
    assert sum(plan.sizes) < sum(R.Plan(probs).sizes)
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for _ in range(6):
        plan.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(plan, i, o)


def test_band_64x64_sampled_walkers():
    R = _R()
    p = R.Problem(L=64, n_windows=64, walkers_per_window=4, k_final=20, interval=100_000, seed=7)
    _say("case: band layout, 64x64 REWL 64x4, X=1e5, 2 intervals")
    plan = R.Plan([p], _band(R))
    dense = R.plan_bytes([p], R.LAYOUT_DENSE)
    assert sum(plan.sizes) < 0.6 * dense
    plan.init()
    plan.run(2)
    o = _oracle_of(p)
    o.run(2)
    compare(plan, 0, o, walkers=[0, 1, 2, 3, 127, 128, 252, 255])
    compare(plan, 0, o, tables=False)
