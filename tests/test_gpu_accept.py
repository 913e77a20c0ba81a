"""The sweep's acceptance decision is the specified FP64 comparison (Eq. 1 in
fixed point), on the device, near the decision boundary.

The sweep decides with a single-precision estimate of exp(x) and falls back to
the FP64 exp_spec comparison only when u lies within 1e-4 of that estimate; its
soundness rests on the float estimate's error bound.  The library's self-check
kernel (not part of the public header) evaluates both decisions on 10^7 pairs
(delta, u) per K, within 1e-3 relative of the boundary and one in eight at the
boundary word itself, and one in sixteen far below it (x <= -23, down to the
largest ln g the layout holds), where the filter rejects with no range test;
it counts disagreements, which must be zero.  A sample of the pairs is also
decided by the CPU oracle, which must agree.
"""
import ctypes as C

import numpy as np
import pytest

from oracle.rewl import accept as oracle_accept

pytestmark = pytest.mark.gpu


def _selfcheck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_02748_amd as R
    f = R.lib().rewl_selfcheck_accept
    f.argtypes = [C.c_int32, C.c_uint64, C.c_int64, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_int32, C.c_int32]
    f.restype = C.c_int
    return R, f


@pytest.mark.parametrize("K,packed", [(6, 0), (20, 0), (40, 0), (6, 1), (20, 1), (24, 1)])
def test_float_filter_never_disagrees_with_the_fp64_comparison(K, packed):
    """packed = 1: the form used with packed table words, where the difference arrives in units
    of 2^-(K + 26) with its low 26 bits clear and is converted to float from its two halves."""
    R, f = _selfcheck()
    n, ns = 10_000_000, 4000
    counts = np.zeros(3, np.int64)
    sd = np.zeros(ns, np.int64)
    su = np.zeros(ns, np.uint32)
    sdec = np.zeros(ns, np.int32)
    print(f"case: acceptance self-check K={K}, packed={packed}, {n} pairs", flush=True)
    R._check(f(K, 1000 + K + 77 * packed, n, 1e-3, counts.ctypes.data, sd.ctypes.data, su.ctypes.data,
               sdec.ctypes.data, ns, packed))
    disagree, exact, acc = (int(x) for x in counts)
    assert disagree == 0, counts
    assert exact > n // 20, counts            # the exact path is really exercised
    assert n // 10 < acc < 9 * n // 10, counts  # both outcomes occur near the boundary
    cpu = np.array([oracle_accept(int(d), int(u), K) for d, u in zip(sd, su)])
    assert (cpu == (sdec != 0)).all()
