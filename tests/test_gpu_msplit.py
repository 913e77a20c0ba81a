"""Bit-exact parity of the magnetization-window split (the alternative layout of
Sec. 2) between the HIP path and the CPU oracle: windows over m, every energy,
entry walk and exchange overlap in m, tables [e][m - lo]."""
import numpy as np
import pytest

from oracle.rewl import OracleREWL
from tests.test_gpu_parity import _R, _say, compare

pytestmark = pytest.mark.gpu


def _oracle(p):
    o = OracleREWL(p.L, p.n_windows, p.overlap, p.walkers_per_window, p.k_final, p.flat, p.interval,
                   p.seed, p.init, sync=p.stage_sync, split=p.split)
    o.init()
    return o


def test_msplit_4x4_full_run_batched_and_plain():
    R = _R()
    p = R.Problem(L=4, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=10, interval=10_000, seed=2,
                  split=R.SPLIT_MAGNETIZATION)
    _say("case: magnetization split 4x4, 3 windows x 2 walkers, K=10, to the end, batched and plain")
    batched = R.Plan([p], R.Tuning(graph_intervals=8))
    plain = R.Plan([p], R.Tuning(form=R.FORM_PLAIN))
    batched.init()
    plain.init()
    orc = _oracle(p)
    for _ in range(400):
        batched.run(8)
        plain.run(8)
        orc.run(8)
        if orc.info()["done"]:
            break
    assert orc.info()["done"]
    compare(batched, 0, orc)
    compare(plain, 0, orc)
    d = batched.walker(0, 1, 0)
    assert d["lng"].shape == (17, d["hi"] - d["lo"] + 1)


def test_msplit_mixed_lattices_and_rules_prefix():
    R = _R()
    M = R.SPLIT_MAGNETIZATION
    probs = [R.Problem(L=8, n_windows=3, overlap=(3, 4), walkers_per_window=3, k_final=8, interval=1000, seed=31,
                       split=M),
             R.Problem(L=12, n_windows=4, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=32,
                       split=M, stage_sync=R.SYNC_WINDOW),
             R.Problem(L=16, n_windows=5, overlap=(3, 4), walkers_per_window=2, k_final=8, interval=1000, seed=33,
                       split=M)]
    _say("case: magnetization split, L in {8,12,16}, both stage rules, 150 intervals")
    plan = R.Plan(probs, R.Tuning(graph_intervals=5))
    plan.init()
    orcs = [_oracle(p) for p in probs]
    for _ in range(6):
        plan.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(plan, i, o)


def test_msplit_plan_rules_on_host():
    R = _R()
    E, M = R.SPLIT_ENERGY, R.SPLIT_MAGNETIZATION
    with pytest.raises(R.RewlError):
        R.Plan([R.Problem(L=8, split=E), R.Problem(L=8, split=M)])      # one split per plan
    plan = R.Plan([R.Problem(L=8, n_windows=2, overlap=(1, 2), walkers_per_window=2, split=M)])
    plan.init()
    lo, hi = plan.window(0, 1)
    assert (lo, hi) == OracleREWL(8, 2, (1, 2), 2, 20, split=1).window(1)
    assert np.all([lo <= plan.walker(0, 1, a, tables=False)["m"] <= hi for a in range(2)])
