"""ln Z on tensor-product (beta, h) grids (factorised through the M columns)
on the GPU, against the float64 oracle evaluated point by point.

The factorised sums regroup the same positive terms, so ln Z agrees with
the oracle's direct sum to a few ulp per term (1e-10 absolute allowed, as for
the direct kernel).  Moments come from column statistics with the law of total
variance, each a central sum, so the second moments keep ~1e-10 relative
accuracy (1e-8 allowed, absolute floor scaled by N).
"""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import lnz as Z

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_02748_amd as R
    R.lib()
    return torch, R


def _synthetic(L):
    N = L * L
    lge = exact.exact_lngE(L)
    return lge[:, None] + exact.binomial_lng(N)[None, :] - N * math.log(2.0), N


def _tables():
    G4 = exact.enumerate_joint(4)
    with np.errstate(divide="ignore"):
        lng4 = np.where(G4 > 0, np.log(np.maximum(G4, 1)), -np.inf)   # holes inside rows and columns
    lng8, N8 = _synthetic(8)
    noisy = lng8 + np.random.default_rng(3).normal(0, 0.3, lng8.shape)
    noisy[:, 7] = -np.inf                                           # an empty column
    noisy[20, :] = -np.inf                                          # an empty row
    return [(lng4, 16), (lng8, N8), (noisy, N8)]


def _check_moments(mom, ref, b, h, N):
    B, H = np.meshgrid(b, h, indexing="ij")
    want = {0: ref["M"], 1: -ref["E"] + H * ref["M"], 2: ref["varU"], 3: ref["varM"], 4: ref["covUM"]}
    for col, w in want.items():
        got = mom[..., col]
        tol = 1e-8 * np.maximum(np.abs(w), 1.0) + 1e-9 * N
        assert np.all(np.abs(got - w) <= tol), (N, col, np.max(np.abs(got - w)))


@pytest.mark.parametrize("nb,nh", [(1, 1), (13, 5), (9, 300)])
def test_grid_forward_and_moments_against_oracle(nb, nh):
    """Ragged beta blocks (13 = 8 + 5) and more than one chunk of h (300 > 256)."""
    torch, R = _torch()
    b = np.linspace(0.05, 1.3, nb)
    h = np.linspace(-0.7, 0.6, nh)
    for lng, N in _tables():
        dl = torch.tensor(lng, device="cuda")
        db, dh = torch.tensor(b, device="cuda"), torch.tensor(h, device="cuda")
        z = R.lnz_grid_forward(dl, db, dh, N)
        ref = Z.moments(lng, b[:, None], h[None, :])
        assert z.shape == (nb, nh)
        assert np.max(np.abs(z.cpu().numpy() - ref["lnz"])) < 1e-10
        _, _, _, mom = R.lnz_grid_backward(dl, db, dh, z, None, N, want_grads=False, want_mom=True)
        _check_moments(mom.cpu().numpy(), ref, b, h, N)


def test_grid_equals_direct_kernel_on_the_same_points():
    torch, R = _torch()
    lng, N = _synthetic(16)
    b = np.linspace(0.1, 1.0, 40)
    h = np.linspace(-0.5, 0.5, 33)
    B, H = np.meshgrid(b, h, indexing="ij")
    dl = torch.tensor(lng, device="cuda")
    zg = R.lnz_grid_forward(dl, torch.tensor(b, device="cuda"), torch.tensor(h, device="cuda"), N).cpu().numpy()
    zd = R.lnz_forward(dl, torch.tensor(B.ravel(), device="cuda"), torch.tensor(H.ravel(), device="cuda"), N)
    assert np.max(np.abs(zg.ravel() - zd.cpu().numpy())) < 1e-10


def test_grid_sub_table_offsets():
    torch, R = _torch()
    lng, N = _synthetic(8)
    e0, e1, m0, m1 = 5, 50, 3, 60
    sub = np.full_like(lng, -np.inf)
    sub[e0:e1, m0:m1] = lng[e0:e1, m0:m1]
    b, h = np.linspace(0.2, 0.9, 6), np.linspace(-0.3, 0.4, 7)
    dl = torch.tensor(np.ascontiguousarray(lng[e0:e1, m0:m1]), device="cuda")
    z = R.lnz_grid_forward(dl, torch.tensor(b, device="cuda"), torch.tensor(h, device="cuda"), N, e0=e0, m0=m0)
    assert np.max(np.abs(z.cpu().numpy() - Z.lnz(sub, b[:, None], h[None, :]))) < 1e-10


def test_grid_gradients_against_oracle():
    torch, R = _torch()
    lng, N = _tables()[2]
    b, h = np.linspace(0.2, 0.9, 11), np.linspace(-0.4, 0.5, 7)
    go = np.random.default_rng(5).uniform(0.5, 1.5, (11, 7))
    dl = torch.tensor(lng, device="cuda")
    db, dh = torch.tensor(b, device="cuda"), torch.tensor(h, device="cuda")
    z = R.lnz_grid_forward(dl, db, dh, N)
    gb, gh, gl, _ = R.lnz_grid_backward(dl, db, dh, z, torch.tensor(go, device="cuda"), N, want_lng=True)
    rb, rh, rl = Z.grads(lng, b[:, None], h[None, :], go)
    assert np.allclose(gb.cpu().numpy(), rb.sum(1), rtol=1e-9, atol=1e-9)
    assert np.allclose(gh.cpu().numpy(), rh.sum(0), rtol=1e-9, atol=1e-9)
    glc = gl.cpu().numpy()
    assert np.all(glc[~np.isfinite(lng)] == 0.0)
    assert np.allclose(glc, rl, rtol=1e-9, atol=1e-12)


def test_grid_autograd_finite_differences_and_second_derivatives():
    torch, R = _torch()
    LnZG = R.LnZGrid()
    lng, N = _synthetic(6)
    lng = lng + np.random.default_rng(1).normal(0, 0.2, lng.shape)
    dl = torch.tensor(lng, device="cuda", requires_grad=True)
    db = torch.tensor(np.linspace(0.2, 0.8, 4), device="cuda", requires_grad=True)
    dh = torch.tensor(np.linspace(-0.3, 0.3, 3), device="cuda", requires_grad=True)
    f = lambda bb, hh: LnZG.apply(dl.detach(), bb, hh, N)
    assert torch.autograd.gradcheck(f, (db, dh), eps=1e-6, atol=1e-6, rtol=1e-5)
    assert torch.autograd.gradgradcheck(f, (db, dh), eps=1e-5, atol=1e-5, rtol=1e-4)
    g = lambda ll: LnZG.apply(ll, db.detach(), dh.detach(), N)
    small = torch.tensor(lng[:12, :12].copy(), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda ll: LnZG.apply(ll, db.detach(), dh.detach(), N, 0, 0), (small,),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
    del g
    # specific heat and susceptibility on the grid, against the oracle's moments
    lng8, N8 = _synthetic(8)
    b, h = np.linspace(0.2, 0.9, 5), np.linspace(-0.4, 0.4, 4)
    db = torch.tensor(b, device="cuda", requires_grad=True)
    dh = torch.tensor(h, device="cuda", requires_grad=True)
    z = LnZG.apply(torch.tensor(lng8, device="cuda"), db, dh, N8)
    # d/d beta_i of sum_j lnZ(i, j) and d/d h_j of sum_i lnZ(i, j)
    gb, gh = torch.autograd.grad(z.sum(), (db, dh), create_graph=True)
    gbb, = torch.autograd.grad(gb.sum(), (db,), retain_graph=True)
    ghh, = torch.autograd.grad(gh.sum(), (dh,))
    ref = Z.moments(lng8, b[:, None], h[None, :])
    assert np.allclose(gbb.cpu().numpy(), ref["varU"].sum(1), rtol=1e-8)
    assert np.allclose(ghh.cpu().numpy(), (b[:, None] ** 2 * ref["varM"]).sum(0), rtol=1e-8)


def test_full_size_grid_32x32():
    """The measured configuration: 1025 x 1025 bins, 1024 beta x 256 h."""
    torch, R = _torch()
    lng, N = _synthetic(32)
    b = np.linspace(0.1, 1.0, 1024)
    h = np.linspace(-0.5, 0.5, 256)
    dl = torch.tensor(lng, device="cuda")
    db, dh = torch.tensor(b, device="cuda"), torch.tensor(h, device="cuda")
    z = R.lnz_grid_forward(dl, db, dh, N)
    _, _, _, mom = R.lnz_grid_backward(dl, db, dh, z, None, N, want_grads=False, want_mom=True)
    z, mom = z.cpu().numpy(), mom.cpu().numpy()
    pts = [(0, 0), (0, 255), (1, 128), (511, 17), (700, 200), (1023, 0), (1023, 255), (363, 129)]
    bi = np.array([b[i] for i, _ in pts])
    hj = np.array([h[j] for _, j in pts])
    ref = Z.moments(lng, bi, hj)
    zi = np.array([z[i, j] for i, j in pts])
    assert np.max(np.abs(zi - ref["lnz"])) < 1e-9
    mi = np.array([mom[i, j] for i, j in pts])
    assert np.allclose(mi[:, 0], ref["M"], rtol=1e-8, atol=1e-8 * N)
    assert np.allclose(mi[:, 2], ref["varU"], rtol=1e-8)
    assert np.allclose(mi[:, 3], ref["varM"], rtol=1e-8)
    # every grid point: the synthetic table factorises into ln Z(beta, 0) + N ln cosh(beta h)
    lz0 = Z.lnz(lng, b, 0.0 * b)
    expect = lz0[:, None] + N * np.log(np.cosh(b[:, None] * h[None, :]))
    assert np.max(np.abs(z - expect)) < 1e-9 * np.max(np.abs(expect))
    assert np.allclose(mom[..., 3], N / np.cosh(b[:, None] * h[None, :]) ** 2, rtol=1e-8)


def test_grid_second_order_entry_point_against_oracle():
    """rewl_lnz_grid_backward2: per-point d grad_out and the row / column sums of the Hessian products
    (the reductions run on the device), against the oracle evaluated point by point."""
    torch, R = _torch()
    lng, N = _tables()[2]
    b, h = np.linspace(0.2, 0.9, 11), np.linspace(-0.4, 0.5, 7)
    rng = np.random.default_rng(9)
    g = rng.uniform(0.5, 1.5, (11, 7))
    a, c = rng.normal(size=11), rng.normal(size=7)
    T = lambda x: torch.tensor(x, device="cuda")
    dl, db, dh = T(lng), T(b), T(h)
    z = R.lnz_grid_forward(dl, db, dh, N)
    B, H = np.meshgrid(b, h, indexing="ij")
    for aa, cc in ((a, c), (a, None), (None, c)):
        d_go, d_b, d_h = R.lnz_grid_second(dl, db, dh, z, T(g), None if aa is None else T(aa),
                                           None if cc is None else T(cc), N)
        A = np.zeros_like(B) if aa is None else np.broadcast_to(aa[:, None], B.shape)
        Cc = np.zeros_like(B) if cc is None else np.broadcast_to(cc[None, :], B.shape)
        r_go, r_b, r_h = Z.second(lng, B, H, g, A, Cc)
        assert np.allclose(d_go.cpu().numpy(), r_go, rtol=1e-8, atol=1e-8 * N)
        assert np.allclose(d_b.cpu().numpy(), r_b.sum(1), rtol=1e-8, atol=1e-8 * N)
        assert np.allclose(d_h.cpu().numpy(), r_h.sum(0), rtol=1e-8, atol=1e-8 * N)
