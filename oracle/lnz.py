"""Thermodynamic reweighting of a joint DOS, written as its definition (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The joint DOS g(E,M) the paper computes (Sec. 2) gives the partition function
of the Ising model in a field at any inverse temperature beta and field h:

    ln Z(beta, h) = log sum_{(E,M) visited} exp(ln g(E,M) - beta E + beta h M)

(J = 1, energy E = -sum s_i s_j, Zeeman term -h M in the Hamiltonian).  With
p(E,M) = exp(ln g - beta E + beta h M - ln Z):

    d lnZ / d beta   = <-E + h M>           d lnZ / d h = beta <M>
    d lnZ / d ln g   = p(E, M)
    d2 lnZ / d beta2 = Var(E - h M)          d2 lnZ / d h2 = beta^2 Var(M)
    d2 lnZ / d beta dh = <M> + beta Cov(-E + h M, M)

so the specific heat per spin is beta^2 Var(E - hM) / N and the susceptibility
per spin is beta Var(M) / N.  Every function below evaluates these sums
directly, one grid point at a time, with a max-shifted exponential sum.
"""
import numpy as np


def axes(N):
    """Energy and magnetization of bin (e, m): E = 4e - 2N, M = 2m - N."""
    e = np.arange(N + 1, dtype=np.float64)
    return 4.0 * e - 2.0 * N, 2.0 * e - N


def _terms(lng, N, beta, h):
    E, M = axes(N)
    return lng + (-beta * E)[:, None] + (beta * h * M)[None, :]


def lnz(lng, beta, h):
    """ln Z at each grid point; lng (N+1, N+1) float64 with -inf = unvisited."""
    N = lng.shape[0] - 1
    beta = np.atleast_1d(np.asarray(beta, np.float64))
    h = np.atleast_1d(np.asarray(h, np.float64))
    out = np.empty(np.broadcast(beta, h).shape)
    for i, (b, hh) in enumerate(np.broadcast(beta, h)):
        x = _terms(lng, N, b, hh)
        mx = np.max(x)
        out.flat[i] = mx + np.log(np.sum(np.exp(x - mx)))
    return out


def moments(lng, beta, h):
    """Per grid point: dict of <E>, <M>, Var(E - hM), Var(M), Cov(-E + hM, M), lnZ."""
    N = lng.shape[0] - 1
    E, M = axes(N)
    beta = np.atleast_1d(np.asarray(beta, np.float64))
    h = np.atleast_1d(np.asarray(h, np.float64))
    shape = np.broadcast(beta, h).shape
    res = {k: np.empty(shape) for k in ("lnz", "E", "M", "varU", "varM", "covUM")}
    EE = np.broadcast_to(E[:, None], lng.shape)
    MM = np.broadcast_to(M[None, :], lng.shape)
    for i, (b, hh) in enumerate(np.broadcast(beta, h)):
        x = _terms(lng, N, b, hh)
        mx = np.max(x)
        w = np.exp(x - mx)
        z = np.sum(w)
        p = w / z
        U = -EE + hh * MM           # d(exponent)/d beta
        mE, mM, mU = np.sum(p * EE), np.sum(p * MM), np.sum(p * U)
        res["lnz"].flat[i] = mx + np.log(z)
        res["E"].flat[i] = mE
        res["M"].flat[i] = mM
        res["varU"].flat[i] = np.sum(p * (U - mU) ** 2)
        res["varM"].flat[i] = np.sum(p * (MM - mM) ** 2)
        res["covUM"].flat[i] = np.sum(p * (U - mU) * (MM - mM))
    return res


def grads(lng, beta, h, grad_out=None):
    """Vector-Jacobian products of lnZ w.r.t. beta, h and ln g for upstream grad_out."""
    mo = moments(lng, beta, h)
    beta_b = np.broadcast_to(np.asarray(beta, np.float64), mo["lnz"].shape)
    h_b = np.broadcast_to(np.asarray(h, np.float64), mo["lnz"].shape)
    go = np.ones(mo["lnz"].shape) if grad_out is None else np.asarray(grad_out, np.float64)
    g_beta = go * (-mo["E"] + h_b * mo["M"])
    g_h = go * beta_b * mo["M"]
    N = lng.shape[0] - 1
    g_lng = np.zeros_like(lng)
    for i, (b, hh) in enumerate(zip(beta_b.flat, h_b.flat)):
        x = _terms(lng, N, b, hh)
        g_lng += go.flat[i] * np.exp(x - mo["lnz"].flat[i])
    return g_beta, g_h, g_lng


def second(lng, beta, h, grad_out=None, up_beta=None, up_h=None):
    """Backward of the first-order products (g_beta, g_h) = (g <U>, g beta <M>).

    With upstream gradients a (of g_beta) and c (of g_h), per grid point:
        d grad_out = a <U> + c beta <M>
        d beta     = g (a Var(U) + c (<M> + beta Cov(U, M)))
        d h        = g (a (<M> + beta Cov(U, M)) + c beta^2 Var(M))
    i.e. the Hessian of ln Z in (beta, h) applied to (a, c), times g, and
    the gradient (a, c) . (d lnZ/d beta, d lnZ/d h)."""
    mo = moments(lng, beta, h)
    shape = mo["lnz"].shape
    b = np.broadcast_to(np.asarray(beta, np.float64), shape)
    hh = np.broadcast_to(np.asarray(h, np.float64), shape)
    g = np.ones(shape) if grad_out is None else np.asarray(grad_out, np.float64)
    a = np.zeros(shape) if up_beta is None else np.asarray(up_beta, np.float64)
    c = np.zeros(shape) if up_h is None else np.asarray(up_h, np.float64)
    mU = -mo["E"] + hh * mo["M"]
    cross = mo["M"] + b * mo["covUM"]
    d_go = a * mU + c * b * mo["M"]
    d_beta = g * (a * mo["varU"] + c * cross)
    d_h = g * (a * cross + c * b * b * mo["varM"])
    return d_go, d_beta, d_h
