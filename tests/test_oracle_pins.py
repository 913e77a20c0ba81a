"""Pins of oracle functions that a plausible mistake could otherwise slip past.

* Flatness (Sec. 2, 80 % rule of Sec. 3, read as flat_den * min H * n_seen >=
  flat_num * sum H over the bins the walker has ever visited, ln g > 0): an
  exact tie is flat and one count less is not; never-visited bins are ignored;
  a bin visited in an earlier stage but not in this one (ln g > 0, H = 0)
  keeps the walker from being flat.  Planted mistakes this catches: a strict
  '>' at the tie, the visited set taken from H > 0.
* The random walker matching of an exchange round (Sec. 2, walker pairs chosen
  at random): a Fisher-Yates shuffle must give every one of the W! matchings
  with equal probability (chi-square over 10^5 rounds for W = 3 and 4).  A
  Sattolo shuffle (j < i) gives only the (W-1)! cyclic ones; other off-by-one
  index errors skew the counts.
* The matching point of Eq. (3)-(4) (Sec. 2: where the derivatives of the
  pieces' ln g(E) agree best): on constructed pieces with a known unique
  minimum of |beta_i - beta_j|, with an exact tie (the lowest E wins), and
  with a minimum below the previous matching point (the search starts at the
  previous matching point).  Catches: arg max, forward instead of central
  differences, the tie going up, the search ignoring the previous point, the
  shift applied with the wrong sign.  Every value is a small dyadic rational,
  so the arithmetic is exact and the ties are exact.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import merge as MG
from oracle.rewl import OracleREWL, draw_matching


# ----------------------------------------------------------------- flatness
def _flat_case(lng, H, flat=(4, 5)):
    o = OracleREWL(4, 1, (3, 4), 1, 8, flat, 100, 0)
    shape = o.walker(0)["lng"].shape
    L_ = np.zeros(shape, np.int64)
    H_ = np.zeros(shape, np.uint64)
    for (i, j), v in lng.items():
        L_[i, j] = v
    for (i, j), v in H.items():
        H_[i, j] = v
    o.set_walker(0, lng=L_)
    o.set_hist(0, H_)
    return o.is_flat(0)


def _bins(n):
    return [(3 + k // 5, 2 + 3 * (k % 5)) for k in range(n)]


def test_flatness_exact_tie_is_flat_and_one_less_is_not():
    b = _bins(5)
    seen = {x: 7 for x in b}
    # 5 bins: H = 16, 21, 21, 21, 21 -> sum 100, 5 * 16 * 5 = 400 = 4 * 100: exactly 80 %
    tie = dict(zip(b, [16, 21, 21, 21, 21]))
    assert _flat_case(seen, tie)
    assert not _flat_case(seen, dict(zip(b, [15, 21, 21, 21, 21])))   # min one less
    assert not _flat_case(seen, dict(zip(b, [16, 22, 21, 21, 21])))   # sum one more
    assert _flat_case(seen, dict(zip(b, [17, 21, 21, 21, 21])))       # min one more
    # other thresholds: 100 % needs all equal, 0 % is always flat once anything was seen
    assert _flat_case(seen, dict(zip(b, [9] * 5)), flat=(1, 1))
    assert not _flat_case(seen, dict(zip(b, [9, 9, 9, 9, 10])), flat=(1, 1))
    assert _flat_case(seen, dict(zip(b, [0, 1, 0, 0, 0])), flat=(0, 1))


def test_flatness_counts_only_bins_ever_visited():
    b = _bins(7)
    seen = {x: 7 for x in b[:5]}
    tie = dict(zip(b[:5], [16, 21, 21, 21, 21]))
    # bins never visited (ln g = 0, H = 0) do not count
    assert _flat_case(seen, tie)
    # a bin visited in an earlier stage (ln g > 0) but not yet in this one (H = 0)
    # is part of the visited set: min H = 0, not flat
    seen2 = dict(seen)
    seen2[b[5]] = 3
    assert not _flat_case(seen2, tie)
    # nothing visited at all is not flat
    assert not _flat_case({}, {})


# ----------------------------------------------------------------- matching
@pytest.mark.parametrize("W,rounds", [(3, 100_000), (4, 120_000)])
def test_exchange_matching_is_uniform_over_all_matchings(W, rounds):
    from scipy.stats import chi2
    perms = {p: i for i, p in enumerate(itertools.permutations(range(W)))}
    counts = np.zeros(len(perms), np.int64)
    for r in range(rounds):
        counts[perms[draw_matching(12345, r, r % 5, W)]] += 1
    assert (counts > 0).all(), counts           # every matching occurs (Sattolo reaches only cycles)
    exp = rounds / len(perms)
    stat = float(((counts - exp) ** 2 / exp).sum())
    p = chi2.sf(stat, len(perms) - 1)
    assert p > 1e-4, (stat, p, counts)


def test_exchange_matching_pairs_each_walker_once():
    for W in (1, 2, 5, 8):
        for r in range(50):
            assert sorted(draw_matching(7, r, 3, W)) == list(range(W))


# ----------------------------------------------------------------- matching point
N_ = 64
COL = 32


def _f(e):
    return -((e - 32.0) ** 2) / 128.0 + 20.0


def _bump(e, c):
    return (e - c) ** 2 / 128.0


def _piece(lo, hi, vals, axis="e"):
    t = np.full((hi - lo + 1, N_ + 1), -np.inf)
    t[:, COL] = vals
    return (lo, hi, t) if axis == "e" else (lo, hi, np.ascontiguousarray(t.T))


def _three_pieces(axis="e"):
    e0 = np.arange(0, 41, dtype=np.float64)
    e1 = np.arange(10, 51, dtype=np.float64)
    e2 = np.arange(20, 61, dtype=np.float64)
    p0 = _piece(0, 40, _f(e0), axis)
    p1 = _piece(10, 50, _f(e1) + _bump(e1, 35) + 3.75, axis)
    p2 = _piece(20, 60, _f(e2) + _bump(e2, 35) + _bump(e2, 25) - 2.25, axis)
    expect = np.full(N_ + 1, -np.inf)
    ee = np.arange(0, 61, dtype=np.float64)
    # below 35 from piece 0; from 35 on piece 2 shifted to agree with the joined marginal at 35
    expect[:61] = np.where(ee < 35, _f(ee), _f(ee) + _bump(ee, 35) + _bump(ee, 25) - 100.0 / 128.0)
    return [p0, p1, p2], expect


def _same_up_to_constant(got, want):
    ok = np.isfinite(want)
    assert (np.isfinite(got) == ok).all()
    d = got[ok] - want[ok]
    assert np.max(np.abs(d - d[0])) < 1e-12, d


def test_matching_point_unique_minimum_and_previous_point_rule():
    # pair (0, 1): |beta_0 - beta_1| = |e - 35| / 256, unique minimum at 35.
    # pair (1, 2): over the whole overlap the minimum would be 30 (and 34 is
    # better than 35), but the search starts at the previous matching point 35,
    # where the joined marginal's slope is closest: 35 again.
    pieces, expect = _three_pieces("e")
    joint, marg, emats = MG.merge(pieces, N_, "ground")
    assert emats == [35, 35]
    _same_up_to_constant(joint[:, COL], expect)
    _same_up_to_constant(marg, expect)


def test_matching_point_tie_goes_to_the_lowest_energy():
    e0 = np.arange(0, 41, dtype=np.float64)
    e1 = np.arange(10, 51, dtype=np.float64)
    # |beta_0 - beta_1| = |2e - 61| / 512: equal at e = 30 and e = 31
    pieces = [_piece(0, 40, _f(e0)), _piece(10, 50, _f(e1) + _bump(e1, 30.5) + 1.5)]
    _, _, emats = MG.merge(pieces, N_, "sum")
    assert emats == [30]


def test_magnetization_matching_point_same_rules():
    pieces, expect = _three_pieces("m")
    joint, _, mmats = MG.merge_m(pieces, N_, "sum")
    assert mmats == [35, 35]
    _same_up_to_constant(joint[COL, :], expect)


def test_two_coordinate_join_uses_both_matching_points():
    # one magnetization column joined along E (the three energy pieces), and the
    # three magnetization pieces of one energy row joined along M
    pe, expect_e = _three_pieces("e")
    rects = [(lo, hi, 0, N_, t) for lo, hi, t in pe]
    joint, _, (e_mats, m_mats) = MG.merge_2d(rects, N_, "sum")
    assert e_mats == [[35, 35]] and m_mats == []
    _same_up_to_constant(joint[:, COL], expect_e)
    pm, expect_m = _three_pieces("m")
    rects = [(0, N_, lo, hi, t) for lo, hi, t in pm]
    joint, _, (e_mats, m_mats) = MG.merge_2d(rects, N_, "sum")
    assert m_mats == [35, 35] and e_mats == [[], [], []]
    _same_up_to_constant(joint[COL, :], expect_m)
