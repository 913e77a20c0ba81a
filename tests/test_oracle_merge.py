"""Pins of the oracle's walker averaging and error bars (oracle/merge.py)."""
import math

import numpy as np

from oracle import exact
from oracle import merge as MG


def _frags(rng, W=4, nE=6, nM=9, K=10):
    """Integer fixed-point tables with ragged visit patterns (some bins seen by 0..W walkers)."""
    base = rng.normal(5.0, 1.0, (nE, nM))
    frags = []
    for a in range(W):
        v = np.round((base + rng.normal(0, 0.05, base.shape) + 3.0 * a) * 2 ** K).astype(np.int64)
        seen = rng.random(base.shape) < 0.8
        seen[:2, :2] = True                       # a common region for the alignment
        frags.append(np.where(seen, v, 0))
    return frags, K


def test_error_is_the_leave_one_walker_out_jackknife():
    rng = np.random.default_rng(11)
    frags, K = _frags(rng)
    avg, err = MG.window_average(frags, K, with_err=True)
    vals = [f.astype(np.float64) * 2.0 ** -K for f in frags]
    seen = [f > 0 for f in frags]
    common = np.logical_and.reduce(seen)
    shifted = [v - v[common].mean() for v in vals]       # alignment constants held fixed
    for idx in np.ndindex(avg.shape):
        xs = [s[idx] for s, m in zip(shifted, seen) if m[idx]]
        n = len(xs)
        if n == 0:
            assert avg[idx] == -np.inf and np.isnan(err[idx])
            continue
        assert math.isclose(avg[idx], sum(xs) / n, rel_tol=1e-12, abs_tol=1e-12)
        if n < 2:
            assert np.isnan(err[idx])
            continue
        loo = [(sum(xs) - x) / (n - 1) for x in xs]       # leave-one-out means
        m = sum(loo) / n
        jk = math.sqrt((n - 1) / n * sum((y - m) ** 2 for y in loo))
        assert math.isclose(err[idx], jk, rel_tol=1e-9, abs_tol=1e-12)


def test_identical_walkers_have_zero_error_and_shifted_copies_align():
    rng = np.random.default_rng(3)
    frags, K = _frags(rng, W=1)
    f = frags[0]
    # the same table twice, once offset by a constant on every visited bin
    g = np.where(f > 0, f + (7 << K), 0)
    avg, err = MG.window_average([f, g], K, with_err=True)
    vis = f > 0
    assert np.all(err[vis] < 1e-12)
    v = f.astype(np.float64) * 2.0 ** -K
    assert np.allclose(avg[vis], v[vis] - v[vis].mean(), atol=1e-12)


def test_joint_error_rows_come_from_the_window_of_eq4():
    """Each row of the joint error table is the error of the piece Eq. 4 takes that row from."""
    L = 4
    N = L * L
    lge = exact.exact_lngE(L)
    full = lge[:, None] + exact.binomial_lng(N)[None, :] - N * math.log(2.0)
    pieces, errs = [], []
    for j, (lo, hi) in enumerate(((0, 9), (5, 13), (9, 16))):
        pieces.append((lo, hi, full[lo:hi + 1] + 0.3 * j))
        errs.append(np.full((hi - lo + 1, N + 1), float(j + 1)))
    joint, marg, e_mats, jerr = MG.merge(pieces, N, "sum", errs)
    bounds = [0] + e_mats + [N + 1]
    for j in range(3):
        rows = jerr[bounds[j]:bounds[j + 1]]
        assert np.all(rows == j + 1), (j, bounds)
    # the join itself removes the per-piece offsets exactly
    assert np.allclose(joint[np.isfinite(full)], full[np.isfinite(full)], atol=1e-9)
