"""Pins for the oracle's Wang-Landau / REWL iteration (CPU only).

Exact invariants (hold for every trajectory):
  * the cached (E, M) of each walker equals E, M recomputed from its spins;
  * every walker stays inside its energy window;
  * sum over bins of ln g = sum over stages of (trials in stage) * 2^(K-s);
  * sum over bins of H = trials since the current stage began;
  * a walker's visited bins are realizable states (4x4 enumeration).
Stationary distributions of Eq. (1) at negligible ln f, against enumeration:
  * with ln g frozen at 0 every move is accepted, so H(E,M) follows g(E,M)/2^N;
  * with ln g frozen at the exact value the walk is flat in (E,M).
Eq. (2) detailed balance with frozen tables, against its closed form.
Convergence: a full 4x4 run (serial 2D-WL, f_final = exp(2^-16)) visits
exactly the 80 realizable bins and reproduces ln g(E,M) within the
statistical error of the method; an 8x8 2D-REWL run reproduces the exact
marginal (Fig. 5 comparison) within its statistical error.
"""
import numpy as np
import pytest

from oracle import exact
from oracle import merge as MG
from oracle.rewl import OracleREWL, energy


def _check_invariants(o, stage_trials=None):
    N = o.N
    info = o.info()
    for g in range(o.n_walkers):
        d = o.walker(g)
        E, M = energy(d["spins"], o.L)
        assert d["e"] == (E + 2 * N) // 4 and d["m"] == (M + N) // 2
        assert d["lo"] <= d["e"] <= d["hi"]
        if stage_trials is not None:
            expect = sum(n << (o.K - s) for s, n in enumerate(stage_trials))
            assert int(d["lng"].sum()) == expect
            assert int(d["H"].sum()) == stage_trials[info["stage"]]
    return info


def test_invariants_through_stages_4x4():
    o = OracleREWL(4, 1, (3, 4), 1, 16, (4, 5), 10_000, seed=0)
    o.init()
    trials = [0]
    for _ in range(400):
        if o.info()["done"] or len(trials) >= 8:
            break
        s_before = o.info()["stage"]
        o.sweep(o.X)
        trials[s_before] += o.X
        _check_invariants(o, trials)
        o.boundary()
        if o.info()["stage"] != s_before:
            trials.append(0)
    assert len(trials) >= 4


def test_update_lands_on_the_state_after_the_decision():
    # Sec. 2: on accept g and H change at the trial state, on reject at the
    # current one -- either way at the state the walker holds afterwards, so
    # after every trial the walker's bin has been counted in this stage.
    for L, nw, W in ((4, 1, 1), (8, 3, 2)):
        o = OracleREWL(L, nw, (3, 4), W, 16, (4, 5), 10_000, seed=3)
        o.init()
        moved = 0
        prev = None
        for _ in range(400):
            o.sweep(1)
            for g in range(o.n_walkers):
                d = o.walker(g)
                i = (d["e"] - d["lo"], d["m"])
                assert d["H"][i] > 0 and d["lng"][i] > 0
            cur = [(o.walker(g, False)["e"], o.walker(g, False)["m"]) for g in range(o.n_walkers)]
            moved += prev is not None and cur != prev
            prev = cur
        assert moved > 50


def test_invariants_rewl_16x16_prefix():
    o = OracleREWL(16, 8, (3, 4), 4, 20, (4, 5), 10_000, seed=0)
    o.init()
    for _ in range(20):
        o.sweep(o.X)
        _check_invariants(o, [o.walker(0)["t"]])
        o.boundary()
    assert o.info()["stage"] == 0
    # every walker's visited bins are inside its window and the table is nonnegative
    for g in range(o.n_walkers):
        d = o.walker(g)
        assert (d["lng"] >= 0).all()
        assert d["t"] == 20 * o.X


def test_visited_bins_are_realizable_and_complete_4x4():
    G = exact.enumerate_joint(4)
    o = OracleREWL(4, 1, (3, 4), 1, 16, (4, 5), 10_000, seed=0)
    o.init()
    o.run_to_end()
    assert o.info()["done"] and o.info()["stage"] == 16
    d = o.walker(0)
    assert ((d["lng"] > 0) == (G > 0)).all()


def _frozen_walk(lng_exact_scale, trials, seed=5):
    """4x4 walk with ln g frozen (ln f = 2^-40, 1 unit per visit)."""
    G = exact.enumerate_joint(4)
    K = 40
    o = OracleREWL(4, 1, (3, 4), 1, K, (4, 5), trials, seed=seed)
    o.init()
    with np.errstate(divide="ignore"):
        lg = np.where(G > 0, np.log(np.maximum(G, 1)), 0.0) * lng_exact_scale
    o.set_walker(0, lng=np.round(lg * 2.0 ** K).astype(np.int64) + 1)
    o.set_stage(K)
    o.sweep(trials)
    return G, o.walker(0)["H"].astype(np.float64)


def test_eq1_stationary_infinite_temperature():
    # equal ln g everywhere: every flip accepted, visits follow g(E,M) / 2^N
    G, H = _frozen_walk(0.0, 4_000_000)
    p = G / G.sum()
    assert H[G == 0].sum() == 0
    mask = p > 1e-3
    rel = np.abs(H[mask] / H.sum() - p[mask]) / p[mask]
    assert rel.max() < 0.08, rel.max()


def test_eq1_stationary_flat_with_exact_lng():
    # ln g frozen at the exact ln g(E,M): the 2D walk is flat over the 80 bins
    G, H = _frozen_walk(1.0, 4_000_000)
    h = H[G > 0]
    assert H[G == 0].sum() == 0
    assert abs(h.min() / h.mean() - 1) < 0.15 and abs(h.max() / h.mean() - 1) < 0.15, (h.min(), h.max(), h.mean())


def _exchange_pair(delta_units, K=20, rounds=20_000):
    """Two windows x one walker, frozen tables; returns swap frequencies from X and Y."""
    o = OracleREWL(4, 2, (1, 2), 1, K, (4, 5), 10, seed=9)
    o.init()
    lo0, hi0 = o.window(0)
    lo1, hi1 = o.window(1)
    # configurations X (walker 0) and Y (walker 1), both in the overlap [lo1, hi0]
    rng = np.random.default_rng(0)
    confs = {}
    while len(confs) < 2:
        s = rng.choice(np.array([-1, 1], np.int8), size=16)
        E, M = energy(s, 4)
        e = (E + 32) // 4
        if lo1 <= e <= hi0 and (e, M) not in [(k[0], k[1]) for k in confs]:
            confs[(e, M)] = s
    (eX, MX), (eY, MY) = list(confs)
    mX, mY = (MX + 16) // 2, (MY + 16) // 2
    sX, sY = confs[(eX, MX)], confs[(eY, MY)]
    t0 = np.zeros((hi0 - lo0 + 1, 17), np.int64)
    t1 = np.zeros((hi1 - lo1 + 1, 17), np.int64)
    # ln g_0(X) - ln g_0(Y) + ln g_1(Y) - ln g_1(X) = delta_units
    t0[eX - lo0, mX] = 1000 + delta_units
    t0[eY - lo0, mY] = 1000
    t1[eY - lo1, mY] = 1000
    t1[eX - lo1, mX] = 1000
    o.set_walker(0, lng=t0, spins=sX)
    o.set_walker(1, lng=t1, spins=sY)
    n_from = {"XY": 0, "YX": 0}
    n_acc = {"XY": 0, "YX": 0}
    for k in range(rounds):
        state = "XY" if o.walker(0, tables=False)["e"] == eX and \
            o.walker(0, tables=False)["m"] == mX else "YX"
        n_from[state] += 1
        n_acc[state] += o.exchange(2 * k)      # even rounds pair windows (0, 1)
    return n_from, n_acc


@pytest.mark.parametrize("delta", [-(1 << 20), -(3 << 19), 0, 1 << 19])
def test_eq2_detailed_balance(delta):
    K = 20
    n_from, n_acc = _exchange_pair(delta, K=K)
    p_xy = min(1.0, float(np.exp(delta / 2.0 ** K)))
    p_yx = min(1.0, float(np.exp(-delta / 2.0 ** K)))
    for state, p in (("XY", p_xy), ("YX", p_yx)):
        n = n_from[state]
        if n == 0:
            continue
        f = n_acc[state] / n
        sd = np.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(f - p) <= 5 * sd + 1e-12, (state, f, p, n)
    if delta == 0:
        assert n_acc["XY"] == n_from["XY"] and n_acc["YX"] == n_from["YX"]


def test_exchange_requires_overlap():
    o = OracleREWL(4, 2, (1, 2), 1, 20, (4, 5), 10, seed=9)
    o.init()
    lo1, hi1 = o.window(1)
    lo0, hi0 = o.window(0)
    up = np.ones(16, np.int8)                       # e = 0: outside window 1
    o.set_walker(0, spins=up)
    before = [o.walker(g, tables=False)["e"] for g in (0, 1)]
    for k in range(50):
        assert o.exchange(2 * k) == 0
    assert [o.walker(g, tables=False)["e"] for g in (0, 1)] == before


def test_determinism_same_seed_same_trajectory():
    a = OracleREWL(8, 3, (3, 4), 2, 12, (4, 5), 1000, seed=42)
    b = OracleREWL(8, 3, (3, 4), 2, 12, (4, 5), 1000, seed=42)
    a.init(); b.init()
    a.run(300); b.run(300)
    for g in range(6):
        da, db = a.walker(g), b.walker(g)
        assert (da["lng"] == db["lng"]).all() and (da["H"] == db["H"]).all()
        assert (da["spins"] == db["spins"]).all() and da["t"] == db["t"]


def test_c1_full_run_against_enumeration():
    G = exact.enumerate_joint(4)
    o = OracleREWL(4, 1, (3, 4), 1, 16, (4, 5), 10_000, seed=0)
    o.init()
    o.run_to_end()
    joint, marg, _ = MG.merge_oracle_run(o, "sum")
    mask = G > 0
    err = np.abs(joint[mask] - np.log(G[mask]))
    # statistical error of single 2D-WL runs at f_final = exp(2^-16): 0.08-0.12 over seeds 0-5
    assert err.max() < 0.2, err.max()
    assert err.mean() < 0.06, err.mean()
    assert (~np.isfinite(joint[~mask])).all()


def test_c1_mean_over_100_runs_against_enumeration():
    # Averaging 100 independent runs (seeds 0-99) shrinks the statistical error of one run
    # (up to ~0.12 in a bin) tenfold; what stays is the method's residual bias at this ln f,
    # measured at a few 10^-3 (0.008-0.012 worst bin over 200-seed blocks of seeds 0-999).
    # A mistake that tilts the stationary distribution of Eq. (1), in the update or in the
    # merge, shows up here at well below the single-run tolerance: accepting with 0.99 times
    # the Eq. (1) ratio gives max 0.056 / rms 0.022 here but passes the single-run test.
    G = exact.enumerate_joint(4)
    mask = G > 0
    acc = np.zeros(int(mask.sum()))
    for seed in range(100):
        o = OracleREWL(4, 1, (3, 4), 1, 16, (4, 5), 10_000, seed=seed)
        o.init()
        o.run_to_end()
        joint, _, _ = MG.merge_oracle_run(o, "sum")
        acc += joint[mask] - np.log(G[mask])
    mean = acc / 100
    assert np.abs(mean).max() < 0.035, np.abs(mean).max()
    assert np.sqrt((mean ** 2).mean()) < 0.01


@pytest.mark.slow
def test_rewl_8x8_marginal_against_exact():
    ex = exact.exact_lngE(8)
    o = OracleREWL(8, 3, (3, 4), 2, 10, (4, 5), 1000, seed=0)
    o.init()
    o.run_to_end()
    assert o.info()["done"]
    joint, marg, e_mats = MG.merge_oracle_run(o, "sum")
    ok = np.isfinite(ex)
    assert (np.isfinite(marg) == ok).all()
    d = np.abs(marg[ok] - ex[ok])
    assert d.max() < 0.6, d.max()            # edges: single-run WL error at ln f = 2^-10
    eps = MG.relative_error(marg, ex)
    assert np.median(eps) < 0.02, np.median(eps)
