"""Pins for the exact references (brute-force g(E,M) and Kaufman/Beale g(E)).

The exact g(E) is the comparison the paper makes in Sec. 3 (Fig. 5); its
computation is checked here against enumeration, the total count 2^N, the
E -> -E symmetry of the square lattice, and the closed-form counts of the
lowest excitations.  The stored fixtures under tests/golden/ were written by
tests/golden/make_golden.py, which calls only oracle/.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact


def test_enumeration_4x4_joint_support():
    G = exact.enumerate_joint(4)
    assert G.sum() == 2 ** 16
    assert (G > 0).sum() == 80          # realizable (E, M) bins of the 4x4 torus
    # ground states: all up / all down
    assert G[0, 16] == 1 and G[0, 0] == 1 and G[0, 1:16].sum() == 0
    # spin-flip symmetry M -> -M and sublattice symmetry E -> -E
    assert (G == G[:, ::-1]).all()
    assert (G.sum(1) == G.sum(1)[::-1]).all()
    # the interior holes of the E = -16 row (e = 4)
    assert list(G[4]) == [0, 0, 88, 96, 24, 0, 0, 0, 8, 0, 0, 0, 24, 96, 88, 0, 0]
    assert G[5, 8] == 0                 # E = -12, M = 0 is empty


def test_kaufman_equals_enumeration_at_L4():
    G = exact.enumerate_joint(4)
    assert list(exact.exact_gE(4)) == [int(x) for x in G.sum(1)]


@pytest.mark.parametrize("L", [6, 8, 12, 16])
def test_kaufman_closed_form_properties(L):
    N = L * L
    g = exact.exact_gE(L)
    assert sum(g) == 2 ** N
    assert list(g) == list(g[::-1])
    assert g[0] == 2 and g[1] == 0           # E = -2N + 4 is impossible
    assert g[2] == 2 * N                     # one flipped spin
    assert g[3] == 4 * N                     # two neighbouring flipped spins
    assert all(v >= 0 for v in g)


def test_golden_exact_lng_matches(golden_dir):
    with open(os.path.join(golden_dir, "exact_lngE.json")) as f:
        data = json.load(f)
    for key, entry in data["lattices"].items():
        L = int(key)
        if L > 16:
            continue                          # larger L: fixture only (slow to recompute)
        ref = exact.exact_lngE(L)
        got = np.array([(-math.inf if v is None else v) for v in entry["lnge"]])
        fin = np.isfinite(ref)
        assert (np.isfinite(got) == fin).all()
        assert np.allclose(got[fin], ref[fin], rtol=0, atol=1e-12)


def test_support_envelope_against_enumeration_4x4():
    # lowest and highest realizable energy per magnetization, by brute force; the
    # realizable energies fill the range except holes next to m = N/2 only
    from oracle.exact import enumerate_joint, support_envelope
    G = enumerate_joint(4)
    e_min, e_max = support_envelope(4)
    for m in range(17):
        es = np.nonzero(G[:, m])[0]
        assert (es.min(), es.max()) == (e_min[m], e_max[m]), m
        holes = sorted(set(range(e_min[m], e_max[m] + 1)) - set(es.tolist()))
        if abs(m - 8) > 1:
            assert holes == [], (m, holes)
    # the holes of this lattice: one below the top at m = 7, 9; three at m = 8
    assert sorted(set(range(e_min[8], e_max[8] + 1)) - set(np.nonzero(G[:, 8])[0].tolist())) == [5, 14, 15]
