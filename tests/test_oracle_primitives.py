"""Pins for the oracle's building blocks (CPU only).

* Philox4x32-10 against ROCm's independent rocRAND implementation (compiled
  from its public header into a throwaway harness) -- counter-based RNG.
* the acceptance exponential against mpmath, and the acceptance rule against
  an exact rational comparison (Eq. 1 / Eq. 2 in fixed point);
* the window decomposition (Sec. 2, Fig. 1(b); Sec. 3) against its defining
  properties;
* the energy / magnetization of a configuration against a numpy rewrite.
"""
import os
import random
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import rewl as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _harness(tmp_path_factory):
    exe = tmp_path_factory.mktemp("philox") / "harness"
    src = os.path.join(HERE, "philox_ref_harness.cpp")
    compiler = shutil.which("g++") or shutil.which("hipcc")
    if compiler is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header or a C++ compiler is unavailable")
    subprocess.run([compiler, "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    src, "-o", str(exe)], check=True)
    return str(exe)


def test_philox_known_answers(tmp_path_factory):
    exe = _harness(tmp_path_factory)
    rng = random.Random(1508)
    cases = [(0, 0, 0), ((1 << 64) - 1, (1 << 62) - 1, (1 << 64) - 1)]
    for _ in range(300):
        cases.append((rng.getrandbits(64), rng.getrandbits(62), rng.getrandbits(64)))
    # counters of the kind the method uses: small attempt blocks, walker ids, tags
    for t in (0, 1, 2, 12345, (1 << 32) + 7):
        for g in (0, 31, 1 << 20):
            for tag in (0, 1, 2, 3, 4):
                cases.append((0, t, g | ((tag << 24) << 32)))
    inp = "".join(f"{k} {c01} {c23}\n" for k, c01, c23 in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (k, c01, c23), line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        ctr = [c01 & 0xFFFFFFFF, c01 >> 32, c23 & 0xFFFFFFFF, c23 >> 32]
        assert O.philox(k, ctr) == ref, (k, ctr)


def test_philox_zero_block_is_not_trivial():
    w = O.philox(0, [0, 0, 0, 0])
    assert len(set(w)) == 4 and all(x != 0 for x in w)


def test_uniform_range_and_resolution():
    assert O.uniform(0) == 2.0 ** -33
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -33
    for w in (1, 12345, 1 << 31, 0xFFFFFFFE):
        assert Fraction(O.uniform(w)) == (Fraction(w) + Fraction(1, 2)) / 2 ** 32


def test_exp_spec_matches_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 200
    rng = np.random.default_rng(7)
    xs = list(-rng.uniform(0, 23, 4000)) + [-1e-300, -2.0 ** -40, -0.5, -1.0, -22.999999]
    xs += [-k * np.log(2.0) for k in range(1, 34)]          # reduction boundaries
    xs += [-(k + 0.5) * np.log(2.0) for k in range(0, 33)]  # rounding ties of k
    worst = 0.0
    for x in xs:
        got = O.exp_spec(x)
        ref = mp.exp(mp.mpf(x))
        ulp = np.spacing(float(ref))
        worst = max(worst, float(abs(mp.mpf(got) - ref)) / ulp)
    assert worst <= 2.0, worst


def test_exp_spec_exact_points():
    assert O.exp_spec(0.0) == 1.0
    assert O.exp_spec(-0.0) == 1.0
    # monotone over a fine grid (the acceptance probability never inverts)
    xs = np.linspace(-22.999, 0, 20001)
    ys = [O.exp_spec(x) for x in xs]
    assert all(a <= b for a, b in zip(ys, ys[1:]))


def test_accept_rule_against_exact_comparison():
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 200
    rng = random.Random(3)
    K = 20
    for delta in (0, 1, 1 << 40):
        assert O.accept(delta, 0xFFFFFFFF, K)
    assert not O.accept(-(23 << K), 0, K)
    assert not O.accept(-(23 << K) - 1, 0, K)
    # just inside the cut: e^-(23 - 2^-K) is still below the smallest u
    assert not O.accept(-(23 << K) + 1, 0, K)
    n_tie = 0
    for _ in range(3000):
        delta = -rng.randrange(1, 23 << K)
        w = rng.getrandbits(32)
        u = (mp.mpf(w) + mp.mpf(0.5)) / 2 ** 32
        p = mp.exp(mp.mpf(delta) / 2 ** K)
        if abs(u - p) < 1e-14 * p:
            n_tie += 1
            continue
        assert O.accept(delta, w, K) == bool(u < p), (delta, w)
    assert n_tie < 5


@pytest.mark.parametrize("N,n,p,q", [(256, 8, 3, 4), (1024, 16, 3, 4), (4096, 64, 3, 4),
                                     (256, 3, 1, 2), (64, 3, 1, 2), (144, 4, 3, 4), (16, 1, 3, 4)])
def test_windows_cover_overlap_and_are_equal(N, n, p, q):
    ws = [O.window(N, n, p, q, i) for i in range(n)]
    assert ws[0][0] == 0 and ws[-1][1] == N
    widths = [hi - lo for lo, hi in ws]
    for (lo0, hi0), (lo1, hi1) in zip(ws, ws[1:]):
        assert lo0 < lo1 <= hi0 < hi1          # neighbours overlap, order kept
        ov = (hi0 - lo1) / (hi0 - lo0)
        assert abs(ov - p / q) <= 2.0 / (hi0 - lo0) + 1e-12
    if n > 1:
        assert max(widths[:-1]) - min(widths[:-1]) <= 1   # equal-sized (last may be clipped)
    if n == 1:
        assert ws == [(0, N)]


def test_windows_of_the_16x16_problem():
    # 8 windows, 3/4 overlap on e in [0, 256]: D = 11, window i = [floor(256 i/11), ceil(256 (i+4)/11)]
    got = [O.window(256, 8, 3, 4, i) for i in range(8)]
    assert got == [(0, 94), (23, 117), (46, 140), (69, 163), (93, 187), (116, 210),
                   (139, 233), (162, 256)]


def test_energy_magnetization_vs_numpy():
    rng = np.random.default_rng(11)
    for L in (2, 4, 6, 16, 32):
        for _ in range(5):
            s = rng.choice(np.array([-1, 1], np.int8), size=(L, L))
            E = -int((s * np.roll(s, -1, 1)).sum() + (s * np.roll(s, -1, 0)).sum())
            assert O.energy(s, L) == (E, int(s.sum()))
        up = np.ones((L, L), np.int8)
        assert O.energy(up, L) == (-2 * L * L, L * L)
        if L % 2 == 0:
            chk = np.fromfunction(lambda r, c: 1 - 2 * ((r + c) % 2), (L, L)).astype(np.int8)
            assert O.energy(chk, L) == (2 * L * L, 0)
