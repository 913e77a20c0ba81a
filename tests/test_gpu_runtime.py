"""Runtime features through the C ABI: autotuner, tuning changes, checkpoint /
resume.  None may change results: every case ends bit-identical to the oracle."""
import pytest

from tests.test_gpu_parity import _R, _oracle_of, _say, compare

pytestmark = pytest.mark.gpu


def _probs(R, n, **kw):
    base = dict(L=8, n_windows=3, walkers_per_window=4, k_final=10, interval=800)
    base.update(kw)
    return [R.Problem(seed=s, **base) for s in range(n)]


def test_autotune_runs_the_plan_and_keeps_results():
    """The autotuner times its candidates on real intervals of the plan (no copy of the buffers):
    afterwards the plan has advanced by the intervals it ran, exactly as under any fixed tuning."""
    R = _R()
    from paper_1508_02748_amd.tune import autotune
    probs = _probs(R, 300)
    _say("case: autotune on 300 x 12 walkers")
    plan = R.Plan(probs, R.Tuning(graph_intervals=2))
    plan.init()
    plan.run(3)
    best = autotune(plan, intervals=1, candidates=[(64, 0), (128, 2), (256, 4), (64, 8), (64, 0, 16)],
                    use_cache=False, graph_lengths=(1, 3))
    assert best.walkers_per_wg in (64, 128, 256) and best.graph_intervals in (1, 3)
    ran = plan.tune_report["intervals_run"]
    assert ran == 2 * 5 + 2 * 2 * (1 + 3)
    plan.run(3)
    for i in (0, 150, 299):
        o = _oracle_of(probs[i])
        o.run(6 + ran)
        compare(plan, i, o)


def test_set_tuning_midway_keeps_results():
    R = _R()
    probs = _probs(R, 40)
    plan = R.Plan(probs, R.Tuning(graph_intervals=3))
    plan.init()
    plan.run(4)
    plan.set_tuning(R.Tuning(walkers_per_wg=256, graph_intervals=1, grid_waves_per_cu=1))
    plan.run(4)
    o = _oracle_of(probs[7])
    o.run(8)
    compare(plan, 7, o)


def test_checkpoint_resume_is_bit_exact():
    R = _R()
    probs = _probs(R, 5, k_final=6, interval=500)
    _say("case: save after 6 intervals, resume in a new plan")
    a = R.Plan(probs)
    a.init()
    a.run(6)
    blob = a.save()
    a.run(6)
    b = R.Plan(probs)
    b.load(blob)
    b.run(6)
    for i in range(5):
        o = _oracle_of(probs[i])
        o.run(12)
        compare(a, i, o)
        compare(b, i, o)
    c = R.Plan(probs)
    with pytest.raises(R.RewlError):
        c.load(blob[: len(blob) // 2])
    other = R.Plan(_probs(R, 5, k_final=7, interval=500))
    with pytest.raises(R.RewlError):
        other.load(blob)


@pytest.mark.parametrize("form", ["batched", "plain"])
def test_int64_headroom_guard_reports_overflow(form):
    """ln g is int64 in units of 2^-K and every visit at stage s adds 2^(K-s): with K = 40 a walker
    that stays at stage 0 (100 % flatness is never reached) adds 2^40 per trial, and its ln g could
    pass 2^62 after 2^22 trials.  The guard must report REWL_EOVERFLOW at the first boundary whose
    interval would take the bound past 2^62 (interval 5 for 10^6 trials per interval), not before."""
    R = _R()
    X = 1_000_000
    p = R.Problem(L=4, n_windows=1, walkers_per_window=1, k_final=40, flat=(1, 1), interval=X, seed=3)
    tn = R.Tuning(form=R.FORM_PLAIN) if form == "plain" else R.Tuning(graph_intervals=1)
    _say(f"case: int64 headroom guard, K = 40, {form} form")
    plan = R.Plan([p], tn)
    plan.init()
    first_bad = next(k for k in range(1, 100) if k * X * 2 ** 40 > 2 ** 62)
    assert first_bad == 5
    for k in range(1, first_bad):
        plan.run(1)
        q = plan.query()
        assert int(q["stage"][0]) == 0 and int(q["trials"][0]) == k * X
    plan.run(1)
    with pytest.raises(R.RewlError) as ei:
        plan.query()
    assert ei.value.status == R.REWL_EOVERFLOW


def test_destroyed_plan_leaves_no_kernel_writing_freed_memory():
    """rewl_plan_destroy (Plan.close / del) waits for the plan's stream: after a long enqueued run
    and an immediate delete, a tensor that the caching allocator hands the same memory must keep
    what is written into it."""
    import torch
    R = _R()
    probs = _probs(R, 64, interval=200_000)
    plan = R.Plan(probs, R.Tuning(graph_intervals=4))
    plan.init()
    sizes = list(plan.sizes)
    plan.run(8)                      # about a second of enqueued work on the plan's stream
    del plan                         # returns the buffers to the caching allocator
    for n in sizes:
        x = torch.empty(max(1, n), dtype=torch.uint8, device="cuda")
        x.fill_(0x5A)
        torch.cuda.synchronize()
        assert bool((x == 0x5A).all())
