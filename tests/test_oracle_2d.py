"""Pins for windows in both energy and magnetization (the second alternative
layout named at the end of Sec. 2), oracle only (CPU).

The energy windows and the magnetization windows (each the overlapping-window
formula) form a grid of rectangles; a rectangle is kept when it holds a state
by the closed-form support (or_realizable: the lowest energy of k minority
spins is the shortest domain wall around them on the torus, the highest puts
them on one sublattice, and the bins between are realizable except three next
to m = N/2).  A proposal leaving the rectangle is rejected; the entry walk
measures the distance to the rectangle in both coordinates; exchange pairs are
neighbours in E on rounds with bit 1 of r clear and neighbours in M on the
others.  The join runs along E within each magnetization column, then along M.
"""
import math

import numpy as np

from oracle import exact
from oracle import merge as MG
from oracle.rewl import OracleREWL, energy, realizable


def _rect_slice(G, r):
    return G[r[0]:r[1] + 1, r[2]:r[3] + 1]


def test_support_equals_enumeration_4x4():
    G = exact.enumerate_joint(4)
    for e in range(17):
        for m in range(17):
            assert realizable(4, e, m) == (G[e, m] > 0), (e, m)


def test_grid_keeps_exactly_the_rectangles_holding_states():
    G = exact.enumerate_joint(4)
    from oracle.rewl import window
    o = OracleREWL(4, 4, (1, 2), 1, 8, (4, 5), 100, seed=0, split=2, m_windows=(4, (1, 2)))
    kept = {o.window_rect(w) for w in range(o.n_windows)}
    for ie in range(4):
        for im in range(4):
            r = window(16, 4, 1, 2, ie) + window(16, 4, 1, 2, im)
            assert (r in kept) == bool((_rect_slice(G, r) > 0).any()), r
    # at 16 x 16 an 8 x 8 grid loses the corners at high energy and large |M|
    assert OracleREWL(16, 8, (1, 2), 1, 8, (4, 5), 100, split=2, m_windows=(8, (1, 2))).n_windows == 56


def test_2d_invariants_8x8():
    o = OracleREWL(8, 3, (1, 2), 2, 10, (4, 5), 500, seed=6, split=2, m_windows=(3, (1, 2)))
    o.init()
    for k in range(40):
        o.sweep(o.X)
        for g in range(o.n_walkers):
            d = o.walker(g)
            E, M = energy(d["spins"], 8)
            assert (d["e"], d["m"]) == ((E + 128) // 4, (M + 64) // 2)
            r = o.window_rect(g // o.W)
            assert r[0] <= d["e"] <= r[1] and r[2] <= d["m"] <= r[3]
            assert d["lng"].shape == (r[1] - r[0] + 1, r[3] - r[2] + 1)
            assert int(d["lng"].sum()) == d["t"] << (o.K - o.info()["stage"])
        o.boundary()
        o.exchange(k)


def test_2d_full_run_4x4_visits_exactly_the_states_and_matches_enumeration():
    G = exact.enumerate_joint(4)
    mask = G > 0
    o = OracleREWL(4, 3, (1, 2), 2, 14, (4, 5), 10_000, seed=0, split=2, m_windows=(3, (1, 2)))
    o.init()
    o.run_to_end()
    assert o.info()["done"]
    for w in range(o.n_windows):
        seen = (o.walker(2 * w)["lng"] > 0) | (o.walker(2 * w + 1)["lng"] > 0)
        assert (seen == (_rect_slice(G, o.window_rect(w)) > 0)).all(), w
    joint, marg, _ = MG.merge_oracle_run(o, "sum")
    d = np.abs(joint[mask] - np.log(G[mask]))
    # seeds 0-5: max 0.045-0.079, mean 0.013-0.020
    assert d.max() < 0.15 and d.mean() < 0.04, (d.max(), d.mean())
    assert np.isneginf(joint[~mask]).all()


def _pair_frequencies(o, w, v, r0, delta, K, rounds=12_000):
    """walkers of windows w and v (one each) with frozen tables; Eq. (2) on rounds r0 + 4k"""
    rw, rv = o.window_rect(w), o.window_rect(v)
    rng = np.random.default_rng(3)
    confs = {}
    while len(confs) < 2:                    # two configurations inside both rectangles
        s = rng.choice(np.array([-1, 1], np.int8), size=16)
        E, M = energy(s, 4)
        e, m = (E + 32) // 4, (M + 16) // 2
        if all(r[0] <= e <= r[1] and r[2] <= m <= r[3] for r in (rw, rv)) and (e, m) not in confs:
            confs[(e, m)] = s
    (eX, mX), (eY, mY) = list(confs)
    tw = np.zeros((rw[1] - rw[0] + 1, rw[3] - rw[2] + 1), np.int64)
    tv = np.zeros((rv[1] - rv[0] + 1, rv[3] - rv[2] + 1), np.int64)
    tw[eX - rw[0], mX - rw[2]] = 1000 + delta      # ln g_w(X) - ln g_w(Y) + ln g_v(Y) - ln g_v(X)
    tw[eY - rw[0], mY - rw[2]] = 1000
    tv[eY - rv[0], mY - rv[2]] = 1000
    tv[eX - rv[0], mX - rv[2]] = 1000
    o.set_walker(w, lng=tw, spins=confs[(eX, mX)])
    o.set_walker(v, lng=tv, spins=confs[(eY, mY)])
    n_from = {"XY": 0, "YX": 0}
    n_acc = {"XY": 0, "YX": 0}
    for k in range(rounds):
        dw = o.walker(w, tables=False)
        state = "XY" if (dw["e"], dw["m"]) == (eX, mX) else "YX"
        before = (dw["e"], dw["m"])
        n_from[state] += 1
        o.exchange(r0 + 4 * k)
        dw = o.walker(w, tables=False)
        n_acc[state] += (dw["e"], dw["m"]) != before
    return n_from, n_acc


def test_2d_exchange_detailed_balance_in_both_directions():
    K = 20
    # 2 x 2 grid at 4 x 4: windows 0 (low e, low m), 1 (low e, high m), 2 (high e, low m), 3
    for (w, v, r0) in ((0, 2, 0), (0, 1, 2)):            # neighbours in E on r = 0, in M on r = 2
        for delta in (-(1 << 20), 0, 1 << 19):
            o = OracleREWL(4, 2, (1, 2), 1, K, (4, 5), 10, seed=9, split=2, m_windows=(2, (1, 2)))
            o.init()
            n_from, n_acc = _pair_frequencies(o, w, v, r0, delta, K)
            for state, p in (("XY", min(1.0, math.exp(delta / 2.0 ** K))),
                             ("YX", min(1.0, math.exp(-delta / 2.0 ** K)))):
                if n_from[state]:
                    f = n_acc[state] / n_from[state]
                    assert abs(f - p) <= 5 * math.sqrt(max(p * (1 - p), 1e-12) / n_from[state]) + 1e-12, \
                        (w, v, delta, state, f, p)
            if delta == 0:
                assert n_acc == n_from


def test_2d_join_of_exact_pieces_is_exact():
    G = exact.enumerate_joint(4)
    with np.errstate(divide="ignore"):
        lg = np.log(G.astype(np.float64))
    o = OracleREWL(4, 3, (1, 2), 1, 8, (4, 5), 10, split=2, m_windows=(3, (1, 2)))
    pieces = [r + (_rect_slice(lg, r) + 0.75 * w - 3.0,) for w, r in
              enumerate(o.window_rect(w) for w in range(o.n_windows))]
    joint, marg, _ = MG.merge_2d(pieces, 16, "sum")
    ok = G > 0
    assert np.allclose(joint[ok], lg[ok], atol=1e-12)
    assert np.isneginf(joint[~ok]).all()
    assert np.allclose(marg, exact.exact_lngE(4), atol=1e-12)


def test_2d_8x8_marginal_against_exact():
    # 3 x 3 rectangles (overlap 1/2 both ways) x 2 walkers to ln f = 2^-10; seeds 0-2 reach
    # max |d ln g(E)| 0.09-0.23, mean 0.03-0.05
    ex = exact.exact_lngE(8)
    ok = np.isfinite(ex)
    o = OracleREWL(8, 3, (1, 2), 2, 10, (4, 5), 1000, seed=0, split=2, m_windows=(3, (1, 2)))
    o.init()
    o.run_to_end()
    assert o.info()["done"]
    joint, marg, _ = MG.merge_oracle_run(o, "sum")
    assert (np.isfinite(marg) == ok).all()
    d = np.abs(marg[ok] - ex[ok])
    assert d.max() < 0.6 and d.mean() < 0.1, (d.max(), d.mean())
