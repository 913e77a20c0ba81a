"""Pins for the oracle's per-window REWL variant (sync = 1): each window
refines ln f alone once its own walkers are flat, after averaging their ln g
(a common REWL form; the paper's own runs refine all windows together).

  * reduction: with one window and one walker the variant is the paper's
    serial 2D-WL trajectory, bit for bit (averaging one table is the identity;
    only H differs once the run has ended, as the variant clears it);
  * at every boundary a window whose walkers were all flat ends with identical
    tables on all its walkers, each bin between the smallest and the largest
    value its visitors held, unvisited bins untouched, and H cleared; windows
    not all flat keep their stage and their tables;
  * a finished window's walkers make no more trials and take part in no
    exchange; the run ends when every window has ended;
  * a full 4x4 run and an 8x8 run reproduce the exact densities of states
    within the statistical error of the method.
"""
import numpy as np
import pytest

from oracle import exact
from oracle import merge as MG
from oracle.rewl import OracleREWL


def test_one_window_one_walker_reduces_to_the_paper_variant():
    a = OracleREWL(4, 1, (3, 4), 1, 12, (4, 5), 2000, seed=5, sync=0)
    b = OracleREWL(4, 1, (3, 4), 1, 12, (4, 5), 2000, seed=5, sync=1)
    a.init(); b.init()
    for _ in range(60):
        a.run(5); b.run(5)
        da, db = a.walker(0), b.walker(0)
        assert (da["lng"] == db["lng"]).all()
        assert da["t"] == db["t"] and a.info() == b.info()
        if not a.info()["done"]:      # the per-window variant clears H when the window ends
            assert (da["H"] == db["H"]).all()
    assert a.info()["done"]


def test_boundary_averages_exactly_the_windows_that_are_flat():
    o = OracleREWL(8, 3, (1, 2), 3, 8, (4, 5), 500, seed=3, sync=1)
    o.init()
    advanced = 0
    for _ in range(4000):
        if o.info()["done"]:
            break
        o.sweep(o.X)
        before = {g: o.walker(g) for g in range(o.n_walkers)}
        states = [o.window_state(w) for w in range(o.n_windows)]
        flat = {g: bool(o.walker(g)["flag"]) or o.is_flat(g) for g in range(o.n_walkers)}
        o.boundary()
        for w in range(o.n_windows):
            s0, done0 = states[w]
            s1, done1 = o.window_state(w)
            gs = [w * o.W + a for a in range(o.W)]
            if done0:
                assert (s1, done1) == (s0, True)
                for g in gs:
                    assert o.walker(g)["t"] == before[g]["t"]
                continue
            if all(flat[g] for g in gs):
                advanced += 1
                assert (s1 == s0 + 1 and not done1) or (s0 == o.K and done1)
                after = [o.walker(g)["lng"] for g in gs]
                for x in after[1:]:
                    assert (x == after[0]).all()
                stack = np.array([before[g]["lng"] for g in gs])
                vis = stack > 0
                anyv = vis.any(0)
                assert (after[0][~anyv] == 0).all()
                lo = np.where(vis, stack, np.iinfo(np.int64).max).min(0)
                hi = np.where(vis, stack, 0).max(0)
                assert (after[0][anyv] >= lo[anyv]).all() and (after[0][anyv] <= hi[anyv]).all()
                for g in gs:   # H restarts after every averaging, also when the window ends
                    assert int(o.walker(g)["H"].sum()) == 0
            else:
                assert (s1, done1) == (s0, False)
                for g in gs:
                    assert (o.walker(g)["lng"] == before[g]["lng"]).all()
    assert advanced >= 6
    info = o.info()
    assert info["done"] == all(o.window_state(w)[1] for w in range(o.n_windows))


def test_finished_windows_do_not_exchange():
    o = OracleREWL(8, 3, (1, 2), 2, 6, (4, 5), 500, seed=1, sync=1)
    o.init()
    while not o.info()["done"]:
        states = [o.window_state(w)[1] for w in range(o.n_windows)]
        if any(states) and not all(states):
            break
        o.run(1)
    done = [o.window_state(w)[1] for w in range(o.n_windows)]
    assert any(done) and not all(done)
    r = o.info()["boundaries"]
    spins = [o.walker(g)["spins"].copy() for g in range(o.n_walkers)]
    o.sweep(o.X)   # finished windows make no trials
    for w in range(o.n_windows):
        if done[w]:
            for a in range(o.W):
                g = w * o.W + a
                assert (o.walker(g)["spins"] == spins[g]).all()
    for rr in (r, r + 1):  # both parities: no accepted swap may touch a finished window
        before = [o.walker(g)["spins"].copy() for g in range(o.n_walkers)]
        o.exchange(rr)
        for w in range(o.n_windows):
            if done[w]:
                for a in range(o.W):
                    g = w * o.W + a
                    assert (o.walker(g)["spins"] == before[g]).all()


def test_full_4x4_run_two_walkers_against_enumeration():
    G = exact.enumerate_joint(4)
    o = OracleREWL(4, 1, (3, 4), 2, 16, (4, 5), 10_000, seed=0, sync=1)
    o.init()
    o.run_to_end()
    a, b = o.walker(0)["lng"], o.walker(1)["lng"]
    assert (a == b).all()             # the last averaging leaves one table
    joint, marg, _ = MG.merge_oracle_run(o, "sum")
    mask = G > 0
    err = np.abs(joint[mask] - np.log(G[mask]))
    assert err.max() < 0.2, err.max()
    assert (~np.isfinite(joint[~mask])).all()


@pytest.mark.slow
def test_rewl_8x8_per_window_marginal_against_exact():
    ex = exact.exact_lngE(8)
    o = OracleREWL(8, 3, (1, 2), 3, 10, (4, 5), 1000, seed=0, sync=1)
    o.init()
    o.run_to_end()
    assert o.info()["done"]
    joint, marg, e_mats = MG.merge_oracle_run(o, "sum")
    ok = np.isfinite(ex)
    assert (np.isfinite(marg) == ok).all()
    d = np.abs(marg[ok] - ex[ok])
    assert d.max() < 0.6, d.max()
    eps = MG.relative_error(marg, ex)
    assert np.median(eps) < 0.02, np.median(eps)
