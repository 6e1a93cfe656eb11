"""Reference solution of P(N) with bounds on the inputs, wlo_t <= w_t <= whi_t
(the inequality-constrained problem of Sec. 3 whose Newton steps P(N)
gives).

Test infrastructure only (see the package docstring).

Plain definition, no interior-point method: the dynamics are eliminated
(x = T w + z0 by forward simulation of the unit inputs), the objective
becomes 1/2 w'Hw + g'w over the stacked inputs, and the bound-constrained
minimiser is found by bounded-variable least squares (scipy's lsq_linear,
method "bvls", an active-set method that terminates at the exact minimiser)
on 1/2 |L'w + L^{-1} g|^2 with H = L L'.
"""
import numpy as np
from scipy.optimize import lsq_linear

from . import kkt


def condense(prob):
    """Returns (T, z0, H, g, const-free): x (stacked (N+1) nx) = Tx w + x0c and
    the reduced Hessian / gradient in w (stacked N nu)."""
    nx, nu, N = kkt.dims(prob)
    Qxw = kkt._get(prob, "Qxw", (N, nx, nu))
    a, lx, lw = kkt._get(prob, "a", (N, nx)), kkt._get(prob, "lx", (N, nx)), kkt._get(prob, "lw", (N, nu))
    lN = kkt._get(prob, "lN", (nx,))
    A, B = prob["A"], prob["B"]
    nw = N * nu
    Tx = np.zeros(((N + 1) * nx, nw))
    xc = np.zeros((N + 1) * nx)
    xc[:nx] = prob["x0"]
    for t in range(N):
        rt, rn = slice(t * nx, (t + 1) * nx), slice((t + 1) * nx, (t + 2) * nx)
        Tx[rn] = A[t] @ Tx[rt]
        Tx[rn, t * nu:(t + 1) * nu] += B[t]
        xc[rn] = A[t] @ xc[rt] + a[t]
    H = np.zeros((nw, nw))
    g = np.zeros(nw)
    for t in range(N):
        Xt, xt = Tx[t * nx:(t + 1) * nx], xc[t * nx:(t + 1) * nx]
        E = np.zeros((nu, nw))
        E[:, t * nu:(t + 1) * nu] = np.eye(nu)
        Qx, Qw, S = prob["Qx"][t], prob["Qw"][t], Qxw[t]
        H += Xt.T @ Qx @ Xt + Xt.T @ S @ E + E.T @ S.T @ Xt + E.T @ Qw @ E
        g += Xt.T @ (Qx @ xt + lx[t]) + E.T @ (S.T @ xt + lw[t])
    XN, xN = Tx[N * nx:], xc[N * nx:]
    H += XN.T @ prob["QxN"] @ XN
    g += XN.T @ (prob["QxN"] @ xN + lN)
    return Tx, xc, 0.5 * (H + H.T), g


def solve(prob, wlo, whi):
    """Minimiser of P(N) with wlo <= w <= whi (arrays (N, nu), +-inf allowed).
    Returns dict x ((N+1), nx), w (N, nu) and the reduced gradient."""
    nx, nu, N = kkt.dims(prob)
    Tx, xc, H, g = condense(prob)
    L = np.linalg.cholesky(H)
    rhs = -np.linalg.solve(L, g)
    lo, hi = np.asarray(wlo, dtype=np.float64).reshape(-1), np.asarray(whi, dtype=np.float64).reshape(-1)
    res = lsq_linear(L.T, rhs, bounds=(lo, hi), method="bvls", tol=1e-15, lsmr_tol=None, max_iter=10000)
    w = res.x
    return dict(x=(Tx @ w + xc).reshape(N + 1, nx), w=w.reshape(N, nu), grad=(H @ w + g).reshape(N, nu))
