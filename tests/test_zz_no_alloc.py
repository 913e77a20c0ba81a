"""The no-allocation tensor-product ln Z forward (library-held scratch array)
against the allocating entry point: the same kernels on the same inputs, so
the results must be bit-identical.  Two calls in a row, the second smaller,
so the second call reuses the scratch array that the first one left filled;
and a grid too large for the array is refused before any device work."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import exact

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_02748_amd as R
    R.lib()
    return torch, R


def _table(L):
    N = L * L
    lge = exact.exact_lngE(L)
    lng = lge[:, None] + exact.binomial_lng(N)[None, :] - N * math.log(2.0)
    lng = lng + np.random.default_rng(L).normal(0, 0.05, lng.shape)
    lng[:, 3] = -np.inf                      # an empty column
    return lng, N


def _pair(torch, R, lng, N, nb, nh, e0=0, m0=0):
    dev = "cuda:0"
    dl = torch.tensor(lng, device=dev)
    b = torch.tensor(np.linspace(0.15, 0.95, nb), device=dev)
    h = torch.tensor(np.linspace(-0.4, 0.45, nh), device=dev)
    ref = R.lnz_grid_forward(dl, b, h, N, e0, m0)
    out = torch.full((nb, nh), float("nan"), dtype=torch.float64, device=dev)
    print(f"case: no-allocation grid forward, table {lng.shape}, grid {nb} x {nh}", flush=True)
    R.lnz_grid_forward_noalloc(dl, b, h, out, N, e0, m0)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_equals_allocating_entry_point_twice():
    torch, R = _torch()
    big, N = _table(32)                           # 1025 x 1025 bins
    got, ref = _pair(torch, R, big, N, 1024, 256)
    assert np.array_equal(got, ref)
    assert np.isfinite(got).all()
    small, n = _table(8)                          # second call: a smaller table and grid
    sub = np.ascontiguousarray(small[4:50, 2:60])
    got2, ref2 = _pair(torch, R, sub, n, 37, 5, e0=4, m0=2)
    assert np.array_equal(got2, ref2)


def test_noalloc_refuses_a_grid_beyond_the_array():
    torch, R = _torch()
    lng, N = _table(32)
    dl = torch.tensor(lng, device="cuda:0")
    limit = 64 << 20
    nb = limit // (8 * lng.shape[1]) + 1          # one row of A too many
    b = torch.linspace(0.1, 1.0, nb, dtype=torch.float64, device="cuda:0")
    h = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    out = torch.empty((nb, 2), dtype=torch.float64, device="cuda:0")
    with pytest.raises(R.RewlError) as ei:
        R.lnz_grid_forward_noalloc(dl, b, h, out, N)
    assert ei.value.status == R.REWL_EINVAL
