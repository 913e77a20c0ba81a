"""Device-side merge (Eq. 3, E_mat, Eq. 4, normalisation) against oracle/merge.py.

Both sides start from bit-identical ln g tables (the sampling is bit-exact), so
differences come only from float64 rounding order: the alignment means (an
exact integer sum on the device, numpy's pairwise sum in the oracle) and the
log-sum-exp reductions, each a few ulp of values below ~1e4, so ln g agrees to
~1e-11 absolute (1e-9 allowed).  Matching points are compared exactly.
"""
import numpy as np
import pytest

from oracle import exact
from oracle import merge as MG
from oracle.rewl import OracleREWL

pytestmark = pytest.mark.gpu


def _R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_02748_amd as R
    R.lib()
    return R


def _pair(R, p, n_intervals, tuning=None):
    plan = R.Plan([p], tuning)
    plan.init()
    plan.run(n_intervals)
    mw = (p.m_windows, p.m_overlap) if p.split == 2 else None
    o = OracleREWL(p.L, p.n_windows, p.overlap, p.walkers_per_window, p.k_final, p.flat, p.interval,
                   p.seed, p.init, split=p.split, m_windows=mw)
    o.init()
    o.run(n_intervals)
    return plan, o


def _points_2d(o, rem):
    """The oracle's (E_mat lists per column, M_mat list) in the device's order: per window its E_mat
    within its column (-1 for the column's lowest window), then the M_mats."""
    e_mats, m_mats = rem
    rects = [o.window_rect(w) for w in range(o.n_windows)]
    cols = sorted({(r[2], r[3]) for r in rects})
    out = [None] * o.n_windows
    for c, key in enumerate(cols):
        members = sorted((r[0], w) for w, r in enumerate(rects) if (r[2], r[3]) == key)
        for k, (_, w) in enumerate(members):
            out[w] = -1 if k == 0 else e_mats[c][k - 1]
    return out + list(m_mats)


def _check(plan, o, norm):
    j, g, em, err = plan.merge(0, norm, with_err=True)
    j, g, err = j.cpu().numpy(), g.cpu().numpy(), err.cpu().numpy()
    rj, rg, rem, rerr = MG.merge_oracle_run(o, norm, with_err=True)
    if getattr(o, "split", 0) == 2:
        rem = _points_2d(o, rem)
    assert em == rem, (em, rem)
    # error bars: NaN exactly where fewer than two walkers visited, else equal to ~1e-12
    assert (np.isnan(err) == np.isnan(rerr)).all()
    ok = ~np.isnan(rerr)
    assert np.max(np.abs(err[ok] - rerr[ok]), initial=0.0) < 1e-9
    fin = np.isfinite(rj)
    assert (np.isfinite(j) == fin).all()
    assert np.max(np.abs(j[fin] - rj[fin])) < 1e-9
    gf = np.isfinite(rg)
    assert (np.isfinite(g) == gf).all()
    assert np.max(np.abs(g[gf] - rg[gf])) < 1e-9
    return j, g


@pytest.mark.parametrize("norm", ["ground", "sum"])
def test_merge_8x8_rewl_matches_oracle(norm):
    R = _R()
    p = R.Problem(L=8, n_windows=3, walkers_per_window=2, k_final=8, interval=1000, seed=2)
    plan, o = _pair(R, p, 300)
    _check(plan, o, norm)


def test_merge_16x16_prefix_matches_oracle():
    R = _R()
    p = R.Problem(L=16, n_windows=8, walkers_per_window=4, k_final=20, interval=10_000, seed=0)
    plan, o = _pair(R, p, 120)
    _check(plan, o, "sum")


def test_merge_single_window_4x4_full_run():
    R = _R()
    p = R.Problem(L=4, n_windows=1, walkers_per_window=1, k_final=16, interval=10_000, seed=0)
    plan, o = _pair(R, p, 400)
    assert o.info()["done"]
    j, g = _check(plan, o, "sum")
    G = exact.enumerate_joint(4)
    mask = G > 0
    assert (np.isfinite(j) == mask).all()
    assert np.max(np.abs(j[mask] - np.log(G[mask]))) < 0.2


@pytest.mark.parametrize("norm", ["ground", "sum"])
def test_merge_magnetization_split_matches_oracle(norm):
    """The join along M (M_mat from the marginals over E) of magnetization windows, dense and band."""
    R = _R()
    p = R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=4,
                  split=R.SPLIT_MAGNETIZATION)
    for lay in (R.LAYOUT_DENSE, R.LAYOUT_BAND):
        plan, o = _pair(R, p, 300, R.Tuning(table_layout=lay))
        _check(plan, o, norm)


def test_merge_16x16_magnetization_split():
    R = _R()
    p = R.Problem(L=16, n_windows=6, overlap=(1, 2), walkers_per_window=3, k_final=12, interval=10_000, seed=8,
                  split=R.SPLIT_MAGNETIZATION)
    plan, o = _pair(R, p, 150)
    _check(plan, o, "sum")


@pytest.mark.parametrize("norm", ["ground", "sum"])
def test_merge_windows_in_both_coordinates(norm):
    """The two-step join of rectangles: along E within each magnetization column, then the columns
    along M; matching points, joint table, marginal and error bars against the oracle."""
    R = _R()
    p = R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=2, k_final=8, interval=1000, seed=6,
                  split=R.SPLIT_BOTH, m_windows=3, m_overlap=(1, 2))
    plan, o = _pair(R, p, 400)
    _check(plan, o, norm)


def test_merge_energy_band_layout():
    R = _R()
    p = R.Problem(L=16, n_windows=8, walkers_per_window=4, k_final=20, interval=10_000, seed=0)
    plan, o = _pair(R, p, 120, R.Tuning(table_layout=R.LAYOUT_BAND))
    _check(plan, o, "sum")
