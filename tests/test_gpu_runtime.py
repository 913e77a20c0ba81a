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


def _first_audit_failure(p, a, max_intervals):
    """Boundary (1-based) at which the audit of the 32-bit stage counts must stop the run: the first
    whose pre-boundary histogram (oracle) holds a bin with 2^(a+1) visits in the current stage.
    With interval = 2^a every boundary audits every walker.  None if the run ends first."""
    o = _oracle_of(p)
    for k in range(1, max_intervals + 1):
        if o.info()["done"]:
            return None, o, k - 1
        o.sweep(p.interval)
        hs = [o.walker(g)["H"] for g in range(o.n_walkers)
              if not o.window_state(g // p.walkers_per_window)[1]]
        if hs and max(int(h.max()) for h in hs) >= 2 ** (a + 1):
            return k, o, k
        o.boundary()
    return None, o, max_intervals


@pytest.mark.parametrize("form,layout", [("batched", 0), ("plain", 0), ("batched", 2), ("plain", 3)])
def test_stage_count_audit_stops_the_run_where_a_count_reaches_the_limit(form, layout):
    """The stage visit counts are kept modulo 2^32 (a 32-bit stage base per bin).  An audit at the
    first boundary after each 2^a stage trials stops the run once some bin has 2^(a+1) visits in
    one stage, which keeps every count below 2^32.  With a = 4, 16-trial intervals and a stage
    that never ends (100 % flatness), the run must stop at exactly the boundary the oracle's
    histogram predicts, and not before."""
    R = _R()
    a = 4
    p = R.Problem(L=4, n_windows=1, walkers_per_window=2, k_final=10, flat=(1, 1), interval=2 ** a, seed=3)
    first, _, _ = _first_audit_failure(p, a, 1000)
    assert first is not None and first > 10
    tn = (R.Tuning(form=R.FORM_PLAIN, audit_shift=a, table_layout=layout) if form == "plain"
          else R.Tuning(graph_intervals=1, audit_shift=a, table_layout=layout))
    _say(f"case: stage-count audit, a = {a}, {form} form, layout {layout}, expected stop at boundary {first}")
    plan = R.Plan([p], tn)
    plan.init()
    for k in range(1, first):
        plan.run(1)
        plan.query()
    plan.run(1)
    with pytest.raises(R.RewlError) as ei:
        plan.query()
    assert ei.value.status == R.REWL_EOVERFLOW


@pytest.mark.parametrize("layout", [0, 3])
def test_stage_count_audit_restarts_with_each_stage(layout):
    """Counts restart at every stage change (new stage base, audit epoch back to zero): at a = 7 no
    stage of this run gives a bin 256 visits, though the walkers make ~40,000 trials each, and the
    run ends bit-exact with the oracle; at a = 6 it stops where the oracle's histogram first
    reaches 128 visits in one stage."""
    R = _R()
    base = dict(L=4, n_windows=2, overlap=(1, 2), walkers_per_window=2, k_final=6, flat=(1, 2), seed=5)
    p7 = R.Problem(interval=2 ** 7, **base)
    first, o, k_end = _first_audit_failure(p7, 7, 5000)
    assert first is None and o.info()["done"]
    _say(f"case: stage-count audit a = 7, run to its end ({k_end} intervals)")
    plan = R.Plan([p7], R.Tuning(graph_intervals=4, audit_shift=7, table_layout=layout))
    plan.init()
    plan.run(k_end + 3)
    compare(plan, 0, o)
    p6 = R.Problem(interval=2 ** 6, **base)
    first, _, _ = _first_audit_failure(p6, 6, 5000)
    assert first is not None
    _say(f"case: stage-count audit a = 6, expected stop at boundary {first}")
    plan = R.Plan([p6], R.Tuning(graph_intervals=1, audit_shift=6, table_layout=layout))
    plan.init()
    plan.run(first - 1)
    plan.query()
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
