"""Pins for the oracle's reweighting ln Z(beta, h) and its derivatives (CPU).

* 4x4: ln Z from the exact joint DOS equals the direct sum over all 65,536
  configurations of exp(-beta E + beta h M).
* closed form: for ln g(E,M) = ln g_exact(E) + ln C(N, m) - N ln 2,
  ln Z = ln Z_0(beta) + N ln cosh(beta h), <M> = N tanh(beta h),
  Var(M) = N / cosh^2(beta h); ln Z_0 is independent of h.
* derivatives: central finite differences of ln Z reproduce the analytic
  first and second derivatives returned by ``moments`` / ``grads``.
"""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import lnz as Z


def _exact_joint(L):
    G = exact.enumerate_joint(L)
    with np.errstate(divide="ignore"):
        return np.where(G > 0, np.log(np.maximum(G, 1)), -np.inf)


def test_lnz_4x4_equals_direct_configuration_sum():
    lng = _exact_joint(4)
    idx = np.arange(1 << 16)
    s = (2 * ((idx[:, None] >> np.arange(16)) & 1) - 1).reshape(-1, 4, 4)
    E = -(s * np.roll(s, -1, 2)).sum((1, 2)) - (s * np.roll(s, -1, 1)).sum((1, 2))
    M = s.sum((1, 2))
    for beta, h in [(0.1, 0.0), (0.4407, 0.0), (1.0, 0.3), (0.7, -0.5), (2.5, 0.05)]:
        x = -beta * E + beta * h * M
        direct = x.max() + math.log(np.exp(x - x.max()).sum())
        assert abs(Z.lnz(lng, beta, h)[0] - direct) < 1e-12 * abs(direct) + 1e-13


def _synthetic(L):
    N = L * L
    lge = exact.exact_lngE(L)
    return lge[:, None] + exact.binomial_lng(N)[None, :] - N * math.log(2.0), N


@pytest.mark.parametrize("L", [4, 8])
def test_lnz_closed_form_synthetic(L):
    lng, N = _synthetic(L)
    betas = np.array([0.2, 0.44, 0.9])
    for b in betas:
        z0 = Z.lnz(lng, b, 0.0)[0]
        for h in (-0.5, -0.1, 0.0, 0.25, 0.5):
            got = Z.lnz(lng, b, h)[0]
            assert abs(got - (z0 + N * math.log(math.cosh(b * h)))) < 1e-10 * abs(got)
            mo = Z.moments(lng, b, h)
            assert abs(mo["M"][0] - N * math.tanh(b * h)) < 1e-9 * N
            assert abs(mo["varM"][0] - N / math.cosh(b * h) ** 2) < 1e-8 * N


def test_first_and_second_derivatives_by_finite_differences():
    lng, N = _synthetic(4)
    lng = lng + np.random.default_rng(0).normal(0, 0.3, lng.shape)   # break the factorisation
    d = 1e-5
    for b, h in [(0.3, 0.2), (0.6, -0.4), (0.44, 0.0)]:
        mo = Z.moments(lng, b, h)
        f = lambda bb, hh: Z.lnz(lng, bb, hh)[0]
        gb = (f(b + d, h) - f(b - d, h)) / (2 * d)
        gh = (f(b, h + d) - f(b, h - d)) / (2 * d)
        assert abs(gb - (-mo["E"][0] + h * mo["M"][0])) < 1e-6 * max(1, abs(gb))
        assert abs(gh - b * mo["M"][0]) < 1e-6 * max(1, abs(gh))
        dd = 1e-4
        gbb = (f(b + dd, h) - 2 * f(b, h) + f(b - dd, h)) / dd ** 2
        ghh = (f(b, h + dd) - 2 * f(b, h) + f(b, h - dd)) / dd ** 2
        assert abs(gbb - mo["varU"][0]) < 1e-3 * max(1, abs(gbb))
        assert abs(ghh - b * b * mo["varM"][0]) < 1e-3 * max(1, abs(ghh))
        gbh = (f(b + dd, h + dd) - f(b + dd, h - dd) - f(b - dd, h + dd) + f(b - dd, h - dd)) / (4 * dd * dd)
        assert abs(gbh - (mo["M"][0] + b * mo["covUM"][0])) < 1e-3 * max(1, abs(gbh))


def test_grad_lng_is_the_probability_table():
    lng, N = _synthetic(4)
    gb, gh, gl = Z.grads(lng, np.array([0.3, 0.5]), np.array([0.1, -0.2]), np.array([1.0, 2.0]))
    assert abs(gl[np.isfinite(lng)].sum() - 3.0) < 1e-12
    # finite difference on one bin
    b, h = 0.3, 0.1
    i, j = 5, 7
    d = 1e-6
    lp, lm = lng.copy(), lng.copy()
    lp[i, j] += d
    lm[i, j] -= d
    fd = (Z.lnz(lp, b, h)[0] - Z.lnz(lm, b, h)[0]) / (2 * d)
    _, _, g1 = Z.grads(lng, b, h)
    assert abs(fd - g1[i, j]) < 1e-7


def _onsager(beta):
    """Onsager's free energy of the infinite square lattice: lim ln Z / N at h = 0."""
    import math
    from scipy.integrate import quad
    k = 2.0 * math.sinh(2.0 * beta) / math.cosh(2.0 * beta) ** 2
    integ = quad(lambda p: math.log((1.0 + math.sqrt(max(0.0, 1.0 - (k * math.sin(p)) ** 2))) / 2.0),
                 0.0, math.pi / 2.0, limit=200, epsabs=1e-14, epsrel=1e-14)[0]
    return math.log(2.0 * math.cosh(2.0 * beta)) + integ / math.pi


@pytest.mark.parametrize("L", [16, 32])
def test_lnz_of_the_exact_tables_against_onsager(L):
    """ln Z(beta, 0) / N of the stored exact g(E) (tests/golden; times the binomial in M) against
    Onsager's infinite-lattice result: equal away from beta_c = 0.4407 up to
    finite-size terms that are exponentially small in L, plus ln 2 / N in the
    ordered phase (the finite lattice counts both ordered states)."""
    import json
    import math
    import os
    N = L * L
    with open(os.path.join(os.path.dirname(__file__), "golden", "exact_lngE.json")) as f:
        lge = np.array([-np.inf if v is None else v for v in json.load(f)["lattices"][str(L)]["lnge"]])
    lng = lge[:, None] + exact.binomial_lng(N)[None, :] - N * math.log(2.0)
    for beta, tol in ((0.1, 1e-12), (0.2, 1e-9), (0.3, 1e-6 if L == 16 else 1e-10)):
        assert abs(float(Z.lnz(lng, beta, 0.0)[0]) / N - _onsager(beta)) < tol, (L, beta)
    for beta in (0.6, 0.8, 1.0):
        d = float(Z.lnz(lng, beta, 0.0)[0]) / N - _onsager(beta)
        assert abs(d - math.log(2.0) / N) < 1e-9, (L, beta, d)


def test_second_order_products_against_finite_differences():
    """Z.second is the Hessian of ln Z in (beta, h) applied to the upstream (a, c), times g, plus the
    gradient dotted with (a, c); every entry checked against finite differences of ln Z itself, so a
    dropped cross term, a wrong power of beta or a swapped upstream fails."""
    lng, N = _synthetic(4)
    lng = lng + np.random.default_rng(3).normal(0, 0.3, lng.shape)
    f = lambda bb, hh: Z.lnz(lng, bb, hh)[0]
    d, dd = 1e-5, 1e-4
    for b, h, g, a, c in [(0.3, 0.2, 1.3, 0.7, -0.4), (0.6, -0.4, 0.5, -1.1, 0.9), (0.44, 0.0, 2.0, 0.0, 1.0)]:
        gb = (f(b + d, h) - f(b - d, h)) / (2 * d)
        gh = (f(b, h + d) - f(b, h - d)) / (2 * d)
        gbb = (f(b + dd, h) - 2 * f(b, h) + f(b - dd, h)) / dd ** 2
        ghh = (f(b, h + dd) - 2 * f(b, h) + f(b, h - dd)) / dd ** 2
        gbh = (f(b + dd, h + dd) - f(b + dd, h - dd) - f(b - dd, h + dd) + f(b - dd, h - dd)) / (4 * dd * dd)
        d_go, d_b, d_h = Z.second(lng, b, h, g, a, c)
        assert abs(d_go[0] - (a * gb + c * gh)) < 1e-6 * max(1, abs(d_go[0]))
        assert abs(d_b[0] - g * (a * gbb + c * gbh)) < 2e-3 * max(1, abs(d_b[0]))
        assert abs(d_h[0] - g * (a * gbh + c * ghh)) < 2e-3 * max(1, abs(d_h[0]))
