"""Windows in both energy and magnetization (the second alternative layout of
Sec. 2) on the device, bit-exact against the CPU oracle: the kept rectangles
(closed-form support), the rectangle window test, the entry distance summed
over both coordinates, exchange between E neighbours and M neighbours on
alternating rounds."""
import pytest

from tests.test_gpu_parity import _R, _oracle_of, _say, compare

pytestmark = pytest.mark.gpu


def _both(R, L, ne, oe, nm, om, **kw):
    return R.Problem(L=L, n_windows=ne, overlap=oe, split=R.SPLIT_BOTH, m_windows=nm, m_overlap=om, **kw)


def test_split2_rectangles_equal_the_oracle():
    R = _R()
    for L, ne, nm in ((4, 2, 2), (8, 3, 3), (16, 8, 8), (12, 5, 2)):
        p = _both(R, L, ne, (1, 2), nm, (1, 2), walkers_per_window=1, k_final=4, interval=100)
        plan = R.Plan([p])
        o = _oracle_of(p)
        assert plan.windows_of[0] == o.n_windows, (L, ne, nm)
        for w in range(o.n_windows):
            assert plan.window_rect(0, w) == o.window_rect(w), (L, w)
    # 16 x 16 with an 8 x 8 grid keeps 56 rectangles
    assert plan.windows_of[0] < ne * nm or L != 16


def test_split2_4x4_full_run_batched_and_plain():
    R = _R()
    p = _both(R, 4, 2, (1, 2), 2, (1, 2), walkers_per_window=2, k_final=8, interval=5000, seed=3)
    _say("case: windows in E and M, 4x4, 2x2 grid x 2 walkers, K=8, to the end")
    batched = R.Plan([p], R.Tuning(graph_intervals=8))
    plain = R.Plan([p], R.Tuning(form=R.FORM_PLAIN))
    batched.init()
    plain.init()
    orc = _oracle_of(p)
    compare(batched, 0, orc)
    for _ in range(400):
        batched.run(8)
        plain.run(8)
        orc.run(8)
        if orc.info()["done"]:
            break
    assert orc.info()["done"]
    compare(batched, 0, orc)
    compare(plain, 0, orc)


def test_split2_8x8_and_16x16_prefix_both_rules():
    R = _R()
    probs = [_both(R, 8, 3, (1, 2), 3, (1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=11),
             _both(R, 8, 3, (3, 4), 2, (1, 2), walkers_per_window=3, k_final=8, interval=1000, seed=12,
                   stage_sync=R.SYNC_WINDOW),
             _both(R, 16, 8, (1, 2), 8, (1, 2), walkers_per_window=1, k_final=8, interval=1000, seed=13, init=1)]
    _say("case: windows in E and M, 8x8 and 16x16 grids, both stage rules, 120 intervals")
    plan = R.Plan(probs, R.Tuning(graph_intervals=4))
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for i, o in enumerate(orcs):
        compare(plan, i, o)
    for _ in range(6):
        plan.run(20)
        for o in orcs:
            o.run(20)
        for i, o in enumerate(orcs):
            compare(plan, i, o)


def test_split2_plan_rules_on_host():
    R = _R()
    with pytest.raises(R.RewlError):           # m_windows without the split
        R.Plan([R.Problem(L=8, m_windows=2, m_overlap=(1, 2))])
    with pytest.raises(R.RewlError):           # the band layout is for one-coordinate splits
        R.Plan([_both(R, 8, 2, (1, 2), 2, (1, 2))], R.Tuning(table_layout=R.LAYOUT_BAND))
    with pytest.raises(R.RewlError):
        R.Plan([_both(R, 8, 2, (1, 2), 0, (1, 2))])
