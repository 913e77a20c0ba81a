"""Pins for the magnetization-window split of the oracle (CPU only).

The paper names splitting the magnetization range, instead of the energy
range, as an alternative layout of the windows (end of Sec. 2).  With
split = 1 every window keeps all energies and a contiguous range of
magnetization bins m = (M + N)/2 given by the same overlapping-window formula;
a proposal leaving the window in m is rejected, the entry walk and the
exchange overlap test use m, and the pieces are joined along M (matching point
M_mat where d ln g(M)/dM of neighbouring pieces agree best).

Pins: exact invariants of the walk; the visited bins of a full 4x4 run are
exactly the realizable (E, M) states of each window; Eq. (2) detailed balance
with frozen tables; the M-join of exact pieces reproduces the exact joint DOS;
a full 4x4 run against enumeration within the method's statistical error.
"""
import math

import numpy as np

from oracle import exact
from oracle import merge as MG
from oracle.rewl import OracleREWL, energy


def _check(o, stage_trials):
    N = o.N
    for g in range(o.n_walkers):
        d = o.walker(g)
        E, M = energy(d["spins"], o.L)
        assert d["e"] == (E + 2 * N) // 4 and d["m"] == (M + N) // 2
        assert d["lo"] <= d["m"] <= d["hi"]                      # inside its m window
        assert d["lng"].shape == (N + 1, d["hi"] - d["lo"] + 1)  # all e x window's m
        expect = sum(n << (o.K - s) for s, n in enumerate(stage_trials))
        assert int(d["lng"].sum()) == expect


def test_msplit_invariants_8x8():
    o = OracleREWL(8, 3, (1, 2), 2, 12, (4, 5), 1000, seed=4, split=1)
    o.init()
    es = set()
    for _ in range(30):
        o.sweep(o.X)
        _check(o, [o.walker(0)["t"]])
        es.update(o.walker(g, tables=False)["e"] for g in range(o.n_walkers))
        o.boundary()
        o.exchange(_)
    assert o.info()["stage"] == 0
    assert len(es) > 10                      # energies are not restricted by the window


def test_msplit_visits_exactly_the_realizable_bins_4x4():
    G = exact.enumerate_joint(4)
    o = OracleREWL(4, 3, (1, 2), 2, 12, (4, 5), 10_000, seed=1, split=1)
    o.init()
    o.run_to_end()
    assert o.info()["done"]
    for w in range(3):
        lo, hi = o.window(w)
        seen = np.zeros((17, hi - lo + 1), bool)
        for a in range(2):
            seen |= o.walker(w * 2 + a)["lng"] > 0
        assert (seen == (G[:, lo:hi + 1] > 0)).all()


def test_msplit_exchange_detailed_balance():
    K = 20
    for delta in (-(1 << 20), 0, 1 << 19):
        o = OracleREWL(4, 2, (1, 2), 1, K, (4, 5), 10, seed=9, split=1)
        o.init()
        lo0, hi0 = o.window(0)
        lo1, hi1 = o.window(1)
        rng = np.random.default_rng(1)
        confs = {}
        while len(confs) < 2:                # two configurations in the m overlap [lo1, hi0]
            s = rng.choice(np.array([-1, 1], np.int8), size=16)
            E, M = energy(s, 4)
            e, m = (E + 32) // 4, (M + 16) // 2
            if lo1 <= m <= hi0 and (e, m) not in confs:
                confs[(e, m)] = s
        (eX, mX), (eY, mY) = list(confs)
        t0 = np.zeros((17, hi0 - lo0 + 1), np.int64)
        t1 = np.zeros((17, hi1 - lo1 + 1), np.int64)
        t0[eX, mX - lo0] = 1000 + delta      # ln g_0(X) - ln g_0(Y) + ln g_1(Y) - ln g_1(X) = delta
        t0[eY, mY - lo0] = 1000
        t1[eY, mY - lo1] = 1000
        t1[eX, mX - lo1] = 1000
        o.set_walker(0, lng=t0, spins=confs[(eX, mX)])
        o.set_walker(1, lng=t1, spins=confs[(eY, mY)])
        n_from = {"XY": 0, "YX": 0}
        n_acc = {"XY": 0, "YX": 0}
        for k in range(20_000):
            w0 = o.walker(0, tables=False)
            state = "XY" if (w0["e"], w0["m"]) == (eX, mX) else "YX"
            n_from[state] += 1
            n_acc[state] += o.exchange(2 * k)
        for state, p in (("XY", min(1.0, math.exp(delta / 2.0 ** K))),
                         ("YX", min(1.0, math.exp(-delta / 2.0 ** K)))):
            if n_from[state]:
                f = n_acc[state] / n_from[state]
                assert abs(f - p) <= 5 * math.sqrt(max(p * (1 - p), 1e-12) / n_from[state]) + 1e-12
        if delta == 0:
            assert n_acc == n_from


def test_msplit_join_of_exact_pieces_is_exact():
    # exact 4x4 ln g cut into three overlapping m windows, each shifted by its
    # own constant: the M-join must undo the shifts exactly (up to rounding)
    G = exact.enumerate_joint(4)
    with np.errstate(divide="ignore"):
        lg = np.log(G.astype(np.float64))
    pieces = []
    for w, c in zip(range(3), (3.25, -7.5, 11.0)):
        o_lo, o_hi = OracleREWL(4, 3, (1, 2), 1, 8, (4, 5), 10, split=1).window(w)
        pieces.append((o_lo, o_hi, lg[:, o_lo:o_hi + 1] + c))
    joint, marg, mm = MG.merge_m(pieces, 16, "sum")
    ok = G > 0
    assert np.allclose(joint[ok], lg[ok], atol=1e-12)
    assert np.isneginf(joint[~ok]).all()
    assert np.allclose(marg, exact.exact_lngE(4), atol=1e-12)
    assert len(mm) == 2 and all(pieces[j + 1][0] <= mm[j] <= pieces[j][1] for j in range(2))


def test_msplit_full_4x4_run_against_enumeration():
    G = exact.enumerate_joint(4)
    ok = G > 0
    for seed in range(3):
        o = OracleREWL(4, 3, (1, 2), 2, 16, (4, 5), 10_000, seed=seed, split=1)
        o.init()
        o.run_to_end()
        assert o.info()["done"]
        joint, marg, _ = MG.merge_oracle_run(o, "sum")
        d = np.abs(joint[ok] - np.log(G[ok]))
        # statistical error of one run at ln f = 2^-16 (max 0.03-0.10, mean 0.009-0.02 over seeds 0-5)
        assert d.max() < 0.15 and d.mean() < 0.03, (seed, d.max(), d.mean())
        assert np.isneginf(joint[~ok]).all()


def test_msplit_8x8_marginal_against_exact():
    # 3 magnetization windows (overlap 3/4) x 2 walkers to ln f = 2^-10: the marginal
    # g(E) = sum_M g(E, M) of the M-joined table against the exact finite-lattice g(E).
    # Seeds 0-2 reach max |d ln g| 0.12-0.22 (the energy split: 0.15-0.35).
    ex = exact.exact_lngE(8)
    ok = np.isfinite(ex)
    o = OracleREWL(8, 3, (3, 4), 2, 10, (4, 5), 1000, seed=0, split=1)
    o.init()
    o.run_to_end()
    assert o.info()["done"]
    joint, marg, m_mats = MG.merge_oracle_run(o, "sum")
    assert (np.isfinite(marg) == ok).all()
    d = np.abs(marg[ok] - ex[ok])
    assert d.max() < 0.6 and d.mean() < 0.1, (d.max(), d.mean())
