"""Packed table words (ln g in bits 63..26, the 26-bit stage base in bits
25..0, 8 bytes per bin) change memory, not results: bit-exact parity with the
CPU oracle in both forms, both stage rules, every split, mixed lattice sizes,
the device merge and checkpoints; and the packed word's own guard, ln g below
2^37 units, stops a run exactly where the oracle's ln g first reaches it."""
import numpy as np
import pytest

from tests.test_gpu_parity import _R, _oracle_of, _say, compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("layout", ["dense_packed", "band_packed"])
def test_packed_16x16_prefix_batched_and_plain(layout):
    R = _R()
    lay = R.LAYOUT_DENSE_PACKED if layout == "dense_packed" else R.LAYOUT_BAND_PACKED
    p = R.Problem(L=16, n_windows=8, walkers_per_window=4, k_final=20, interval=10_000, seed=0)
    _say(f"case: {layout}, 16x16 REWL 8x4, 48 intervals, batched and plain")
    batched = R.Plan([p], R.Tuning(table_layout=lay, graph_intervals=8))
    plain = R.Plan([p], R.Tuning(table_layout=lay, form=R.FORM_PLAIN))
    batched.init()
    plain.init()
    orc = _oracle_of(p)
    for _ in range(3):
        batched.run(16)
        plain.run(16)
        orc.run(16)
        compare(batched, 0, orc)
        compare(plain, 0, orc)


def test_packed_mixed_lattices_stage_rules_to_the_end():
    """Stage changes under the per-window rule at 50 % flatness: the averaging of packed words at
    each window's stage change, and a window that finishes (in the 8x8 problem two of the three
    windows reach stage 6 within the 600 intervals)."""
    R = _R()
    probs = [R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=3, k_final=6, interval=1000, seed=21,
                       stage_sync=R.SYNC_WINDOW, flat=(1, 2)),
             R.Problem(L=12, n_windows=4, walkers_per_window=2, k_final=6, interval=1000, seed=22, flat=(1, 2)),
             R.Problem(L=24, n_windows=6, walkers_per_window=2, k_final=8, interval=1000, seed=23, init=1),
             R.Problem(L=32, n_windows=3, walkers_per_window=2, k_final=8, interval=1000, seed=24,
                       stage_sync=R.SYNC_WINDOW)]
    _say("case: band_packed, L in {8,12,24,32}, both stage rules, 600 intervals")
    plan = R.Plan(probs, R.Tuning(table_layout=R.LAYOUT_BAND_PACKED, graph_intervals=5))
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for _ in range(24):
        plan.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(plan, i, o)
    stages = [orcs[0].window_state(w) for w in range(orcs[0].n_windows)]
    assert max(st for st, _ in stages) >= 2 and any(done for _, done in stages)


@pytest.mark.parametrize("layout", ["dense_packed", "band_packed"])
def test_packed_magnetization_split(layout):
    R = _R()
    lay = R.LAYOUT_DENSE_PACKED if layout == "dense_packed" else R.LAYOUT_BAND_PACKED
    M = R.SPLIT_MAGNETIZATION
    probs = [R.Problem(L=8, n_windows=5, overlap=(1, 2), walkers_per_window=3, k_final=8, interval=1000, seed=31,
                       split=M, flat=(1, 2)),
             R.Problem(L=16, n_windows=8, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=33,
                       split=M, stage_sync=R.SYNC_WINDOW)]
    _say(f"case: {layout}, magnetization split, 150 intervals")
    plan = R.Plan(probs, R.Tuning(table_layout=lay, graph_intervals=5))
    plan.init()
    orcs = [_oracle_of(p) for p in probs]
    for _ in range(6):
        plan.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(plan, i, o)


def test_packed_windows_in_both_coordinates():
    R = _R()
    probs = [R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=6, interval=1000, seed=41,
                       split=R.SPLIT_BOTH, m_windows=3, m_overlap=(1, 2), flat=(1, 2)),
             R.Problem(L=16, n_windows=4, overlap=(1, 2), walkers_per_window=2, k_final=6, interval=1000, seed=42,
                       split=R.SPLIT_BOTH, m_windows=2, m_overlap=(1, 2), stage_sync=R.SYNC_WINDOW)]
    _say("case: dense_packed, windows in both coordinates, 150 intervals, batched and plain")
    batched = R.Plan(probs, R.Tuning(table_layout=R.LAYOUT_DENSE_PACKED, graph_intervals=5))
    plain = R.Plan(probs, R.Tuning(table_layout=R.LAYOUT_DENSE_PACKED, form=R.FORM_PLAIN))
    batched.init()
    plain.init()
    orcs = [_oracle_of(p) for p in probs]
    for _ in range(6):
        batched.run(25)
        plain.run(25)
        for o in orcs:
            o.run(25)
        for i, o in enumerate(orcs):
            compare(batched, i, o)
            compare(plain, i, o)


def test_packed_merge_and_checkpoint_equal_the_unpacked_layout():
    """The device merge reads packed words: on the same 8x8 REWL run it returns the same joint
    ln g, marginal, matching points and errors as with the unpacked band layout; a packed plan
    saved midway and resumed in a new plan ends bit-identical."""
    R = _R()
    p = R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=4, k_final=8, interval=2000, seed=5)
    _say("case: band vs band_packed merge on 8x8 REWL after 200 intervals; packed checkpoint")
    a = R.Plan([p], R.Tuning(table_layout=R.LAYOUT_BAND, graph_intervals=8))
    b = R.Plan([p], R.Tuning(table_layout=R.LAYOUT_BAND_PACKED, graph_intervals=8))
    a.init()
    b.init()
    a.run(100)
    b.run(100)
    blob = b.save()
    a.run(100)
    b.run(100)
    ja, ga, ea, ra = a.merge(0, with_err=True)
    jb, gb, eb, rb = b.merge(0, with_err=True)
    assert ea == eb
    for va, vb in ((ja, jb), (ga, gb), (ra, rb)):
        va, vb = va.cpu().numpy(), vb.cpu().numpy()
        assert va.shape == vb.shape and np.array_equal(va, vb, equal_nan=True)
    unpacked = R.Plan([p], R.Tuning(table_layout=R.LAYOUT_BAND))
    with pytest.raises(R.RewlError):
        unpacked.load(blob)
    c = R.Plan([p], R.Tuning(table_layout=R.LAYOUT_BAND_PACKED, graph_intervals=8))
    c.load(blob)
    c.run(100)
    o = _oracle_of(p)
    o.run(200)
    compare(b, 0, o)
    compare(c, 0, o)


@pytest.mark.parametrize("form", ["batched", "plain"])
def test_packed_ln_g_guard_stops_where_the_oracle_reaches_2_37(form):
    """A packed word holds ln g below 2^37 units.  With K = 24 every stage-0 visit adds 2^24 units,
    so a bin passes 2^37 after 8192 visits; with 100 % flatness the stage never ends.  The run
    must stop (REWL_EOVERFLOW) after exactly the interval in which the oracle's ln g first
    reaches 2^37 in some bin, and not before."""
    R = _R()
    X = 2000
    p = R.Problem(L=4, n_windows=1, walkers_per_window=2, k_final=24, flat=(1, 1), interval=X, seed=9)
    o = _oracle_of(p)
    first = None
    for k in range(1, 2000):
        o.run(1)
        if max(int(o.walker(g)["lng"].max()) for g in range(2)) >= 2 ** 37:
            first = k
            break
    assert first is not None and first > 5
    tn = R.Tuning(table_layout=R.LAYOUT_DENSE_PACKED, graph_intervals=1)
    if form == "plain":
        tn = R.Tuning(table_layout=R.LAYOUT_DENSE_PACKED, form=R.FORM_PLAIN)
    _say(f"case: packed ln g guard, K = 24, {form} form, expected stop after interval {first}")
    plan = R.Plan([p], tn)
    plan.init()
    plan.run(first - 1)
    plan.query()
    o2 = _oracle_of(p)
    o2.run(first - 1)
    compare(plan, 0, o2)
    plan.run(1)
    with pytest.raises(R.RewlError) as ei:
        plan.query()
    assert ei.value.status == R.REWL_EOVERFLOW


@pytest.mark.parametrize("split,layout", [(0, 0), (0, 1), (0, 2), (0, 3), (1, 0), (1, 1), (1, 2), (1, 3), (2, 0),
                                          (2, 2)])
def test_large_batches_every_split_and_layout(split, layout):
    """A batched launch of 16,384 walkers or more whose tables average 2^13 bins per walker or more
    takes the pipelined trial (the next trial's proposal and targets made under the current
    gather); every other launch takes the direct trial, which the small tests here cover.  A
    batch of 32 x 32 problems above both thresholds, in every window split and table layout, with
    both stage rules and with a stage change at every boundary in half of them, against the
    oracle on sampled replicas."""
    R = _R()
    if split == 2:
        base = dict(L=32, n_windows=4, overlap=(1, 2), walkers_per_window=8, k_final=8, interval=1000, split=2,
                    m_windows=4, m_overlap=(1, 2))
    else:
        base = dict(L=32, n_windows=16, overlap=(3, 4), walkers_per_window=8, k_final=8, interval=1000, split=split)
    one = R.Plan([R.Problem(seed=0, **base)], R.Tuning(table_layout=layout))
    per, bins = one.n_walkers, one.sizes[0] // (8 if layout & 2 else 12)
    one.close()
    assert bins >= per << 13, (per, bins)
    n = -(-16384 // per)
    probs = [R.Problem(seed=s, stage_sync=R.SYNC_WINDOW if s % 2 else R.SYNC_PROBLEM,
                       flat=(0, 1) if s % 4 < 2 else (4, 5), **base) for s in range(n)]
    _say(f"case: split {split}, layout {layout}, {n} problems x {per} walkers (pipelined trial), 12 intervals")
    plan = R.Plan(probs, R.Tuning(table_layout=layout, graph_intervals=4))
    assert plan.n_walkers >= 16384
    plan.init()
    plan.run(12)
    for i in (0, 1, 2, n - 1):
        o = _oracle_of(probs[i])
        o.run(12)
        compare(plan, i, o, walkers=[0, 1, per // 2, per - 1])
        compare(plan, i, o, tables=False)
    plan.close()


def test_pipelined_trial_with_small_lattices():
    """Small lattices in a batch that takes the pipelined trial: 16 replicas of the 64 x 64 problem
    (large band tables) lift the batch's average above 2^13 bins per walker, so 1024 8 x 8 problems
    in the same launches run the pipelined trial too.  At 8 x 8 the next proposal reads one of the
    five sites an accepted flip changes in about one accepted trial in thirteen, so its arithmetic
    correction (spin and anti-alignments inverted at the proposal's own site, one anti-alignment
    at a neighbour) runs constantly.  The 8 x 8 problems, with both stage rules and with a stage
    change at every boundary in half of them, against the oracle bit for bit."""
    R = _R()
    big = dict(L=64, n_windows=64, overlap=(3, 4), walkers_per_window=4, k_final=20, interval=1000)
    small = dict(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=4, k_final=8, interval=1000)
    probs = [R.Problem(seed=s, **small, stage_sync=R.SYNC_WINDOW if s % 2 else R.SYNC_PROBLEM,
                       flat=(0, 1) if s % 4 < 2 else (4, 5)) for s in range(1024)]
    probs += [R.Problem(seed=5000 + s, **big) for s in range(16)]
    _say("case: 1024 8x8 problems + 16 64x64 replicas, band packed (pipelined trial), 12 intervals")
    plan = R.Plan(probs, R.Tuning(table_layout=R.LAYOUT_BAND_PACKED, graph_intervals=4))
    bins = plan.sizes[0] // 8
    assert plan.n_walkers >= 16384 and bins >= plan.n_walkers << 13, (plan.n_walkers, bins)
    plan.init()
    plan.run(12)
    for i in (0, 1, 2, 3, 1023):
        o = _oracle_of(probs[i])
        o.run(12)
        compare(plan, i, o)
    plan.close()


@pytest.mark.parametrize("wg,wpw", [(256, 32), (128, 17), (64, 64)])
def test_pipelined_trial_launch_shapes(wg, wpw):
    """The pipelined trial under other launch shapes (fewer walkers per wavefront, smaller
    workgroups, a persistent grid smaller than the batch): a batch of 16 x 16 problems above both
    thresholds gives the oracle's trajectories whatever the shape."""
    R = _R()
    base = dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=10, interval=1000)
    probs = [R.Problem(seed=300 + s, flat=(0, 1) if s % 2 else (4, 5), **base) for s in range(512)]
    _say(f"case: 512 16x16 problems, walkers_per_wg {wg}, walkers_per_wave {wpw} (pipelined trial), 8 intervals")
    plan = R.Plan(probs, R.Tuning(walkers_per_wg=wg, walkers_per_wave=wpw, grid_waves_per_cu=2,
                                  graph_intervals=4))
    bins = plan.sizes[0] // 12
    assert plan.n_walkers >= 16384 and bins >= plan.n_walkers << 13, (plan.n_walkers, bins)
    plan.init()
    plan.run(8)
    for i in (0, 1, 511):
        o = _oracle_of(probs[i])
        o.run(8)
        compare(plan, i, o)
    plan.close()


def test_pipelined_trial_odd_trial_counts():
    """The pipelined trial with odd and tiny trial counts: a walker that starts on the second half
    of a Philox block takes one trial first, the pair loop runs the same count on every lane, and
    one pair or one trial is left; sweeps of 1, 2, 3, 333, 1000 and 7 trials with the boundary work
    between them, on a 16 x 16 batch above both thresholds, against the oracle."""
    R = _R()
    base = dict(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=10, interval=333)
    probs = [R.Problem(seed=700 + s, **base) for s in range(512)]
    _say("case: 512 16x16 problems, odd sweeps of the pipelined trial")
    plan = R.Plan(probs)
    bins = plan.sizes[0] // 12
    assert plan.n_walkers >= 16384 and bins >= plan.n_walkers << 13, (plan.n_walkers, bins)
    plan.init()
    orcs = {i: _oracle_of(probs[i]) for i in (0, 511)}
    for n in (1, 2, 3, 333, 1000, 7):
        plan.sweep(n)
        plan.reduce_lnf()
        plan.exchange()
        for i, o in orcs.items():
            o.sweep(n)
            o.boundary()
            compare(plan, i, o)
    plan.close()
