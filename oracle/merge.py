"""Joining per-walker ln g(E,M) fragments into one joint DOS (Sec. 2, Eq. 3-4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Steps, in the paper's order:

1. Walkers of one window (Sec. 2: several independent walkers per window)
   are combined by aligning each on its mean over the bins all of them have
   visited and averaging ln g where more than one visited a bin (reading of
   the paper's silence on this; the paper only notes that several walkers
   allow error bars, Sec. 2 last paragraph).
2. Marginal over M, Eq. (3): ln g(E) = log sum_M g(E, M).
3. In the overlap of windows i (lower) and j (upper), the inverse
   microcanonical temperature beta(E) = d ln g(E)/dE is taken by central
   differences (ln g(E+4) - ln g(E-4)) / 8 wherever both neighbours exist in
   both pieces; E_mat is the E with the smallest |beta_i - beta_j|, ties to
   the lowest E, searched at or above the previous matching point.
4. Piece j is shifted by one constant, ln g_i(E_mat) - ln g_j(E_mat) of the
   marginals, and Eq. (4) takes piece i below E_mat and piece j from E_mat on.
5. Normalisation: either sum_{E,M} g = 2^N or the ground-state count
   g(E = -2N) = 2.

Error bars (Sec. 2, last paragraph: several walkers per window make error
bars possible): for each bin, the standard error of the window average over
the walkers that visited it, sqrt(sum_a (x_a - mean)^2 / (n (n - 1))) with
x_a the aligned values; this is the jackknife (leave-one-walker-out) error of
that mean with the alignment constants held fixed.  NaN where fewer than two
walkers visited the bin.  The joint table's error in row e is the error of
the window that supplies row e in Eq. (4) (the matching constants are not
counted).

Tables are float64 arrays (N+1, N+1) indexed by (e, m) with -inf where a bin
was never visited; e = (E + 2N)/4, m = (M + N)/2.
"""
import math

import numpy as np


def _lse(a, axis=None):
    a = np.asarray(a, dtype=np.float64)
    mx = np.max(a, axis=axis, keepdims=True)
    mx = np.where(np.isfinite(mx), mx, 0.0)
    with np.errstate(divide="ignore"):
        out = np.log(np.sum(np.exp(a - mx), axis=axis, keepdims=True)) + mx
    return np.squeeze(out, axis=axis) if axis is not None else float(out.reshape(()))


def window_average(frags, K, with_err=False):
    """Step 1: combine the int64 fixed-point tables of one window's walkers.

    frags: list of int64 arrays (n_E, N+1) (units 2^-K; 0 = never visited).
    Returns float64 (n_E, N+1) with -inf on bins no walker visited, and with
    ``with_err`` also the standard error of that average over the walkers."""
    vals = [f.astype(np.float64) * 2.0 ** -K for f in frags]
    seen = [f > 0 for f in frags]
    common = np.logical_and.reduce(seen)
    if not common.any():
        raise ValueError("walkers of a window share no visited bin")
    shifted = [v - v[common].mean() for v in vals]
    num = np.zeros_like(vals[0])
    cnt = np.zeros(vals[0].shape, np.int64)
    for v, s in zip(shifted, seen):
        num[s] += v[s]
        cnt[s] += 1
    out = np.full(vals[0].shape, -np.inf)
    nz = cnt > 0
    out[nz] = num[nz] / cnt[nz]
    if not with_err:
        return out
    ss = np.zeros_like(out)
    for v, s in zip(shifted, seen):
        ss[s] += (v[s] - out[s]) ** 2
    err = np.full(out.shape, np.nan)
    two = cnt > 1
    err[two] = np.sqrt(ss[two] / (cnt[two] * (cnt[two] - 1)))
    return out, err


def marginal(lng_joint):
    """Eq. (3): ln g(E) = log sum_M g(E,M) along the last axis."""
    return _lse(lng_joint, axis=1)


def beta_central(lnge):
    """(ln g(e+1) - ln g(e-1)) / 8 (energy step 4 per bin); nan where undefined."""
    b = np.full(lnge.shape, np.nan)
    ok = np.isfinite(lnge[2:]) & np.isfinite(lnge[:-2]) & np.isfinite(lnge[1:-1])
    b[1:-1][ok] = (lnge[2:][ok] - lnge[:-2][ok]) / 8.0
    return b


def merge(pieces, N, norm="ground", errs=None):
    """Join window pieces into the full joint DOS (Eq. 4).

    pieces: list (ordered by energy) of (lo, hi, lng) with lng float64 of shape
    (hi - lo + 1, N + 1) (-inf = unvisited), already averaged over walkers.
    Returns (lng_joint (N+1, N+1), lng_marginal (N+1,), e_mat list), and with
    ``errs`` (one error table per piece) also the joint error table."""
    full = []
    for lo, hi, t in pieces:
        f = np.full((N + 1, N + 1), -np.inf)
        f[lo:hi + 1] = t
        full.append(f)
    joint = full[0].copy()
    cur_hi = pieces[0][1]
    prev_mat = 0
    e_mats = []
    for j in range(1, len(pieces)):
        lo_j = pieces[j][0]
        gi = marginal(joint)
        gj = marginal(full[j])
        bi, bj = beta_central(gi), beta_central(gj)
        best, e_mat = math.inf, None
        for e in range(max(lo_j, prev_mat), cur_hi + 1):
            if np.isnan(bi[e]) or np.isnan(bj[e]):
                continue
            d = abs(bi[e] - bj[e])
            if d < best:
                best, e_mat = d, e
        if e_mat is None:
            raise ValueError(f"no matching point between pieces {j - 1} and {j}")
        c = gi[e_mat] - gj[e_mat]
        joint[e_mat:] = full[j][e_mat:] + c
        cur_hi = pieces[j][1]
        prev_mat = e_mat
        e_mats.append(e_mat)
    joint = normalise(joint, N, norm)
    if errs is None:
        return joint, marginal(joint), e_mats
    jerr = np.full((N + 1, N + 1), np.nan)
    bounds = [0] + e_mats + [N + 1]
    for j, (lo, hi, _) in enumerate(pieces):
        a, b = max(bounds[j], lo), min(bounds[j + 1], hi + 1)
        if a < b:
            jerr[a:b] = errs[j][a - lo:b - lo]
    return joint, marginal(joint), e_mats, jerr


def merge_m(pieces, N, norm="ground", errs=None):
    """Join magnetization-window pieces (the alternative split of Sec. 2).

    pieces: list (ordered by m) of (lo, hi, lng) with lng float64 of shape
    (N + 1, hi - lo + 1): every energy row, the window's magnetization
    columns.  The same steps as `merge` with the roles of E and M swapped:
    marginal over E, ln g(M) = log sum_E g(E, M); matching point M_mat where
    d ln g(M)/dM of the two pieces agree best; one additive constant per
    piece; the piece below M_mat from the lower window.  Returns (lng_joint
    (N+1, N+1) indexed [e, m], lng_marginal over M (ln g(E)), m_mats[, joint
    error table])."""
    tp = [(lo, hi, np.ascontiguousarray(t.T)) for lo, hi, t in pieces]
    te = None if errs is None else [np.ascontiguousarray(e.T) for e in errs]
    out = merge(tp, N, None, te)
    joint = normalise(np.ascontiguousarray(out[0].T), N, norm)
    res = (joint, marginal(joint), out[2])
    if errs is None:
        return res
    return res + (np.ascontiguousarray(out[3].T),)


def merge_2d(pieces, N, norm="ground", errs=None):
    """Join rectangular (E, M) pieces (windows in both coordinates, Sec. 2 end).

    pieces: list of (e_lo, e_hi, m_lo, m_hi, lng) with lng float64 of shape
    (e_hi - e_lo + 1, m_hi - m_lo + 1), -inf = unvisited.  The pieces of each
    magnetization column (same m range) are first joined along E as energy
    windows (E_mat from ln g(E) = log sum over the column's M), then the
    columns are joined along M (M_mat from ln g(M) = log sum over E).
    Returns (lng_joint (N+1, N+1), ln g(E), (E_mat lists per column, M_mat
    list)), and with ``errs`` (one error table per piece) also the joint error
    table, each bin's error taken from the piece that supplies the bin."""
    cols = {}
    for k, (elo, ehi, mlo, mhi, t) in enumerate(pieces):
        cols.setdefault((mlo, mhi), []).append((elo, ehi, t, None if errs is None else errs[k]))
    col_pieces, col_errs, e_mats = [], [], []
    for (mlo, mhi) in sorted(cols):
        rows, rerr = [], []
        for elo, ehi, t, et in sorted(cols[(mlo, mhi)], key=lambda x: x[0]):
            f = np.full((ehi - elo + 1, N + 1), -np.inf)
            f[:, mlo:mhi + 1] = t
            rows.append((elo, ehi, f))
            if et is not None:
                fe = np.full((ehi - elo + 1, N + 1), np.nan)
                fe[:, mlo:mhi + 1] = et
                rerr.append(fe)
        out = merge(rows, N, None, rerr if errs is not None else None)
        col_pieces.append((mlo, mhi, out[0][:, mlo:mhi + 1]))
        if errs is not None:
            col_errs.append(out[3][:, mlo:mhi + 1])
        e_mats.append(out[2])
    res = merge_m(col_pieces, N, norm, col_errs if errs is not None else None)
    if errs is None:
        return res[0], res[1], (e_mats, res[2])
    return res[0], res[1], (e_mats, res[2]), res[3]


def normalise(joint, N, norm="ground"):
    """Fix the additive constant of ln g: "sum" (sum g = 2^N), "ground" (g(E = -2N) = 2) or None
    (unchanged, for the intermediate joins of the two-coordinate merge)."""
    if norm is None:
        return joint
    if norm == "sum":
        return joint - _lse(joint[np.isfinite(joint)]) + N * math.log(2.0)
    if norm == "ground":
        return joint - marginal(joint)[0] + math.log(2.0)
    raise ValueError(norm)


def relative_error(lnge_sim, lnge_exact):
    """epsilon(E) = |ln g_sim - ln g_exact| / ln g_exact over E with g_exact > 1."""
    ok = np.isfinite(lnge_exact) & (lnge_exact > 0)
    return np.abs(lnge_sim[ok] - lnge_exact[ok]) / lnge_exact[ok]


def merge_oracle_run(orc, norm="ground", with_err=False):
    """Merge all walkers of an OracleREWL simulation into (joint, marginal, e_mats[, joint_err])."""
    pieces, errs = [], []
    for w in range(orc.n_windows):
        frags = [orc.walker(w * orc.W + a)["lng"] for a in range(orc.W)]
        lo, hi = orc.window(w)
        avg, err = window_average(frags, orc.K, with_err=True)
        pieces.append((lo, hi, avg))
        errs.append(err)
    if getattr(orc, "split", 0) == 2:
        rects = [orc.window_rect(w) + (p[2],) for w, p in enumerate(pieces)]
        return merge_2d(rects, orc.N, norm, errs if with_err else None)
    join = merge_m if getattr(orc, "split", 0) else merge
    return join(pieces, orc.N, norm, errs if with_err else None)
