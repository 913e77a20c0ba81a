"""The comparison metrics of the long GPU runs, on the CPU: Eq. (5)'s relative
difference computed from logarithms equals its definition on the densities."""
import numpy as np

from tests.long_convergence import rel_diff


def test_eq5_from_logarithms_equals_definition():
    rng = np.random.default_rng(5)
    a = rng.uniform(-30, 30, 1000)
    b = a + rng.normal(0, 0.5, 1000)
    g1, g2 = np.exp(a), np.exp(b)
    direct = np.abs(g1 - g2) / ((g1 + g2) / 2)
    assert np.allclose(rel_diff(a, b), direct, rtol=1e-12, atol=0)
    assert np.all(rel_diff(a, a) == 0)
    assert np.all(rel_diff(a, b) < 2)              # bounded by 2 when one density vanishes
    assert np.allclose(rel_diff(a, b), rel_diff(b, a))
