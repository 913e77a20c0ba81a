"""Full-size parity through stage changes (the paths behind the measured
configurations): stage advance, the new stage base that restarts H, the
resumable multi-chunk flatness scan, and the headroom bookkeeping, at the
32 x 32, mixed-L and 64 x 64 shapes, in the batched and the plain form and in
both table layouts.

With flatness num/den = 0/1 every walker that has visited a bin is flat at
every boundary, so every boundary advances the stage (Sec. 2: all walkers move
to the next iteration together) and ln f halves each time; the sampled
replicas are compared bit for bit with the oracle after every boundary.  The
16 x 16 problem is also run under the real 80 % rule until both sides have
changed stage twice, with every walker compared at every boundary after the
first stage change."""
import pytest

from tests.test_gpu_parity import _R, _oracle_of, _say, compare

pytestmark = pytest.mark.gpu

C3 = dict(L=32, n_windows=16, overlap=(3, 4), walkers_per_window=8, k_final=24, interval=10_000)
C4 = dict(L=64, n_windows=64, overlap=(3, 4), walkers_per_window=4, k_final=20, interval=100_000)


@pytest.mark.parametrize("layout", [0, 1])
def test_32x32_and_mixed_stage_advance_every_boundary(layout):
    R = _R()
    probs = [R.Problem(seed=300 + s, flat=(0, 1), **C3) for s in range(8)]
    for L, nw in ((8, 2), (12, 4), (16, 8), (24, 12)):
        probs.append(R.Problem(**dict(C3, L=L, n_windows=nw), seed=400 + L, flat=(0, 1)))
    sample = (0, 7, 8, 10, 11)
    _say(f"case: 32x32 x 8 + mixed L, every boundary a stage change, layout {layout}, batched and plain")
    batched = R.Plan(probs, R.Tuning(graph_intervals=3, table_layout=layout))
    batched.init()
    plain = R.Plan([probs[i] for i in sample], R.Tuning(form=R.FORM_PLAIN, table_layout=layout))
    plain.init()
    orcs = {i: _oracle_of(probs[i]) for i in sample}
    for k in range(10):
        batched.run(1)
        plain.run(1)
        for j, i in enumerate(sample):
            orcs[i].run(1)
            ws = [0, 1, 63, 64, 127] if probs[i].L == 32 else None   # a sample of the 128 walkers
            compare(batched, i, orcs[i], walkers=ws)
            compare(plain, j, orcs[i], walkers=ws)
            compare(batched, i, orcs[i], tables=False)
    assert min(o.info()["stage"] for o in orcs.values()) == 10


@pytest.mark.parametrize("layout", [0, 1, 3])
def test_64x64_stage_advance_every_boundary(layout):
    R = _R()
    probs = [R.Problem(seed=500 + s, flat=(0, 1), **C4) for s in range(3)]
    _say(f"case: 64x64 x 3, every boundary a stage change, layout {layout}, 6 boundaries, batched and plain")
    batched = R.Plan(probs, R.Tuning(graph_intervals=2, table_layout=layout))
    batched.init()
    plain = R.Plan(probs[2:], R.Tuning(form=R.FORM_PLAIN, table_layout=layout))
    plain.init()
    o = _oracle_of(probs[2])
    walkers = [0, 1, 2, 3, 64, 127, 128, 200, 252, 253, 254, 255]
    for k in range(6):
        batched.run(1)
        plain.run(1)
        o.run(1)
        compare(batched, 2, o, walkers=walkers)
        compare(plain, 0, o, walkers=walkers)
    compare(batched, 2, o, tables=False)
    assert o.info()["stage"] == 6


@pytest.mark.slow
def test_16x16_real_flatness_through_two_stage_changes(capsys):
    """The 16 x 16 REWL problem (8 windows x 4 walkers, X = 10^4) under a real flatness rule until
    both sides have reached stage 2.  50 % flatness instead of 80 % so that the oracle gets there
    in minutes (about 1.1e4 intervals, 3.6e9 trials; 80 % needs 2.9e4).  Every walker is compared
    after every boundary for 64 boundaries from the first stage change, then every 64 boundaries,
    and again at the second stage change and at the end.  It runs about three minutes, so it
    reports its progress past the output capture."""
    R = _R()
    p = R.Problem(L=16, n_windows=8, overlap=(3, 4), walkers_per_window=4, k_final=20, interval=10_000, seed=0,
                  flat=(1, 2))
    _say("case: 16x16 REWL 8x4, 50% flatness, to stage 2 (oracle ~3 min)")
    plan = R.Plan([p], R.Tuning(graph_intervals=16))
    plan.init()
    o = _oracle_of(p)
    k, first = 0, None
    while o.info()["stage"] < 2:
        step = 1 if first is None or k - first < 64 else 64
        plan.run(step)
        o.run(step)
        k += step
        if first is None and o.info()["stage"] >= 1:
            first = k
            _say(f"first stage change at interval {k}")
        if first is not None:
            compare(plan, 0, o)
        if k % 1024 < step:
            with capsys.disabled():
                print(f"[16x16 real flatness] interval {k}, stage {o.info()['stage']}", flush=True)
        assert k < 20000
    _say(f"stage 2 at interval {k}")
    assert o.info()["stage"] == 2
