"""Exact densities of states of the periodic L x L Ising model (J = 1).

TEST INFRASTRUCTURE ONLY (pins for the oracle, see ``oracle/__init__.py``).

* ``enumerate_joint(L)``: g(E, M) by brute force over all 2^N configurations
  (N = L*L <= 20).  This is the quantity the 2D random walk estimates (Sec. 2).
* ``exact_gE(L)``: the exact g(E) of the finite periodic lattice, the reference
  the paper compares its marginal against (Sec. 1 and Sec. 3, Fig. 5; Beale's
  method).  It is computed from Kaufman's closed form of the torus partition
  function, written as a polynomial in y = exp(-4K):

      x = e^{-2K},  A = (1 + x^2)^2 / (2 x (1 - x^2)),  c_l = A - cos(pi l / L)
      cosh(L gamma_l) = T_L(c_l)            (Chebyshev polynomial)
      Z = 1/2 ((1 - x^2)/x)^{N/2} (Z1 + Z2 + Z3 + Z4)
      Z1 = prod_{r<L/2} (2 T_L(c_{2r+1}) + 2),  Z2 = same with -2
      Z3 = (u0^{L/2} + u0^{-L/2}) (uL^{L/2} + uL^{-L/2}) prod_{1<=r<L/2} (2 T_L(c_{2r}) + 2)
      Z4 = (u0^{L/2} - u0^{-L/2}) (uL^{L/2} - uL^{-L/2}) prod_{1<=r<L/2} (2 T_L(c_{2r}) - 2)
      u0 = (1 - x)/(x (1 + x)),  uL = (1 + x)/(x (1 - x))

  Kaufman's products of 2 cosh(L gamma/2) over l and 2L - l pair up into
  2 T_L(c) + 2, so no square roots remain.  Then x^N Z = sum_j g(-2N + 4j) y^j
  with y = x^2.  The polynomial is evaluated at N + 1 points on a circle in the
  complex plane with mpmath at N + 96 bits, and the coefficients are recovered
  by an inverse discrete Fourier transform and rounded to integers.

* ``support_envelope(L)``: for every magnetization bin, the lowest and highest
  realizable energy bin.  With k = min(m, N - m) minority spins, the fewest
  unsatisfied bonds are those of the shortest closed domain wall around k
  sites on the torus, P_min(k) = min(2 ceil(2 sqrt k), 2L + 2 [L does not
  divide k]) (a compact cluster, or a band wrapping the torus once k >= L),
  and the most are 4k (minority spins on one sublattice, none adjacent), so
  e = P/2 runs from P_min/2 to 2k.  The realizable bins fill this range except
  a few holes next to m = N/2.  The bounds say where windows in both E and M
  hold states.

Both are checked against each other at L = 4, against sum g = 2^N, the E -> -E
symmetry and the counts of the lowest excitations (tests/test_exact.py).
"""
import functools
import math

import numpy as np


def enumerate_joint(L):
    """g(E, M) for the periodic L x L lattice by brute force.

    Returns an int64 array G[e, m] of shape (N+1, N+1), e = (E + 2N)/4 and
    m = (M + N)/2 (the number of up spins)."""
    N = L * L
    if N > 20:
        raise ValueError("enumeration is limited to N <= 20")
    idx = np.arange(1 << N, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(N)) & 1).astype(np.int8)  # site i -> bit i
    s = (2 * bits - 1).reshape(-1, L, L)
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    e = (E + 2 * N) // 4
    m = (M + N) // 2
    G = np.zeros((N + 1, N + 1), np.int64)
    np.add.at(G, (e, m), 1)
    return G


@functools.lru_cache(maxsize=None)
def exact_gE(L):
    """Exact g(E) as a tuple of Python ints indexed by e = (E + 2N)/4, e = 0..N."""
    import mpmath as mp

    if L < 2 or L % 2:
        raise ValueError("L must be even")
    N = L * L
    npts = N + 1
    with mp.workprec(N + 96):
        def P(y):
            x = mp.sqrt(y)
            A = (1 + x * x) ** 2 / (2 * x * (1 - x * x))

            def twoT(l):  # 2 T_L(c_l) = 2 cosh(L * acosh(c_l))
                c = A - mp.cos(mp.pi * l / L)
                return 2 * mp.cosh(L * mp.acosh(c))

            z1 = mp.mpf(1)
            z2 = mp.mpf(1)
            for r in range(L // 2):
                t = twoT(2 * r + 1)
                z1 *= t + 2
                z2 *= t - 2
            z3 = mp.mpf(1)
            z4 = mp.mpf(1)
            for r in range(1, L // 2):
                t = twoT(2 * r)
                z3 *= t + 2
                z4 *= t - 2
            u0 = (1 - x) / (x * (1 + x))
            uL = (1 + x) / (x * (1 - x))
            h = L // 2
            z3 *= (u0 ** h + u0 ** (-h)) * (uL ** h + uL ** (-h))
            z4 *= (u0 ** h - u0 ** (-h)) * (uL ** h - uL ** (-h))
            Z = ((1 - x * x) / x) ** (N // 2) * (z1 + z2 + z3 + z4) / 2
            return x ** N * Z

        # Points y_k = w^(2k+1), w = exp(i pi / npts), avoid y = 1 where
        # (1 - x^2) = 0.  Coefficient j = (1/npts) sum_k P(y_k) w^(-(2k+1) j).
        winv = [mp.expjpi(-mp.mpf(n) / npts) for n in range(2 * npts)]
        ys = [mp.expjpi(mp.mpf(2 * k + 1) / npts) for k in range(npts)]
        vals = [P(y) for y in ys]
        coeffs = []
        for j in range(npts):
            acc = mp.mpc(0)
            for k in range(npts):
                acc += vals[k] * winv[((2 * k + 1) * j) % (2 * npts)]
            coeffs.append(acc / npts)
        out = []
        for c in coeffs:
            v = int(mp.nint(c.real))
            if abs(c.real - v) > 0.25 or abs(c.imag) > 0.25:
                raise ArithmeticError("coefficient not an integer: precision too low")
            out.append(v)
    return tuple(out)


def exact_lngE(L):
    """ln g(E) (float64) indexed by e; -inf where g(E) = 0."""
    g = exact_gE(L)
    return np.array([math.log(v) if v > 0 else -math.inf for v in g])


def binomial_lng(N):
    """ln C(N, m) for m = 0..N (the number of configurations with m up spins)."""
    return np.array([math.lgamma(N + 1) - math.lgamma(m + 1) - math.lgamma(N - m + 1)
                     for m in range(N + 1)])


def support_envelope(L):
    """(e_min, e_max): int arrays over m = 0..N of the lowest and highest
    realizable energy bin at magnetization bin m (see the module notes)."""
    N = L * L
    e_min = np.zeros(N + 1, np.int64)
    e_max = np.zeros(N + 1, np.int64)
    for m in range(N + 1):
        k = min(m, N - m)
        if k == 0:
            p_min = 0
        else:
            p_min = 2 * (math.isqrt(4 * k - 1) + 1)          # 2 ceil(2 sqrt k)
            if k >= L:
                p_min = min(p_min, 2 * L + (0 if k % L == 0 else 2))
        e_min[m] = p_min // 2
        e_max[m] = 2 * k
    return e_min, e_max
