"""The band layout rests on one fact: a state in energy bin e (e = number of
unsatisfied bonds / 2) has at least e/2 minority spins, since every
unsatisfied bond has a minority spin at one end and a spin has four bonds; so
its magnetization bin m lies in [ceil(e/2), N - ceil(e/2)], and with windows in
m the energy bins of a window stay at or below 2 k_max.  Checked here against
exhaustive enumeration at 4 x 4 and against the closed-form support used for
windows in both coordinates at larger L."""
import numpy as np

from oracle import exact
from oracle.rewl import realizable


def test_band_holds_every_state_4x4():
    G = exact.enumerate_joint(4)       # counts by (e, m)
    N = 16
    for e in range(N + 1):
        for m in range(N + 1):
            if G[e, m] > 0:
                lo = (e + 1) // 2
                assert lo <= m <= N - lo, (e, m)
    # the band is tight at its ends for some energies (it is not a loose bound)
    assert G[8, 4] > 0 and G[16, 8] > 0


def test_band_holds_the_closed_form_support():
    for L in (6, 8, 16):
        N = L * L
        for e in range(N + 1):
            lo = (e + 1) // 2
            for m in range(N + 1):
                if realizable(L, e, m):
                    assert lo <= m <= N - lo, (L, e, m)
