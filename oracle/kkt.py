"""KKT system of the UFTOC problem P(N): dense assembly, dense LU solve,
blockwise residual and direct objective evaluation.

Test infrastructure only (see the package docstring).

The paper (Sec. 3) solves P(N) through its KKT system, which it describes as
almost block diagonal; the Riccati recursion is a factorization of it.  Here
the system is written out from the Lagrangian of P(N) (Sec. 2),

    L = sum_t [ 1/2 [x;w]' Q_t [x;w] + l_t' [x;w] + c_t ]
        + 1/2 x_N' QxN x_N + lN' x_N + cN
        + lam_0' (xbar0 - x_0)
        + sum_t lam_{t+1}' (A_t x_t + B_t w_t + a_t - x_{t+1}),

with the unknowns ordered z = (lam_0, x_0, w_0, lam_1, x_1, w_1, ...,
lam_N, x_N).  Its rows are

    lam_0 :  -x_0                                        = -xbar0
    x_t   :  Qx x_t + Qxw w_t - lam_t + A_t' lam_{t+1}    = -lx_t
    w_t   :  Qxw' x_t + Qw w_t + B_t' lam_{t+1}            = -lw_t
    lam_t+1: A_t x_t + B_t w_t - x_{t+1}                   = -a_t
    x_N   :  QxN x_N - lam_N                               = -lN

and the matrix is symmetric.  The multiplier sign is the one that makes
lam_t = P_t x_t - Psi_t (Alg. 3) hold.
"""
import numpy as np


def _get(prob, key, shape):
    v = prob.get(key)
    return np.zeros(shape) if v is None else np.asarray(v, dtype=np.float64)


def dims(prob):
    N, nx = prob["Qx"].shape[0], prob["QxN"].shape[0]
    nu = prob["Qw"].shape[1]
    return nx, nu, N


def _offsets(nx, nu, N):
    """Start index of each block of z: lam_t, x_t (t=0..N), w_t (t<N)."""
    stride = 2 * nx + nu
    lam = [t * stride for t in range(N + 1)]
    xo = [t * stride + nx for t in range(N + 1)]
    wo = [t * stride + 2 * nx for t in range(N)]
    size = N * stride + 2 * nx
    return lam, xo, wo, size


def assemble(prob):
    """Dense KKT matrix K and right-hand side r of P(N)."""
    nx, nu, N = dims(prob)
    lo, xo, wo, size = _offsets(nx, nu, N)
    K = np.zeros((size, size))
    r = np.zeros(size)
    I = np.eye(nx)
    Qxw = _get(prob, "Qxw", (N, nx, nu))
    a, lx = _get(prob, "a", (N, nx)), _get(prob, "lx", (N, nx))
    lw = _get(prob, "lw", (N, nu))
    lN = _get(prob, "lN", (nx,))
    # lam_0 row
    K[lo[0]:lo[0] + nx, xo[0]:xo[0] + nx] = -I
    r[lo[0]:lo[0] + nx] = -np.asarray(prob["x0"])
    for t in range(N):
        X, W, L, Ln = slice(xo[t], xo[t] + nx), slice(wo[t], wo[t] + nu), \
            slice(lo[t], lo[t] + nx), slice(lo[t + 1], lo[t + 1] + nx)
        Xn = slice(xo[t + 1], xo[t + 1] + nx)
        A, B = prob["A"][t], prob["B"][t]
        # x_t row
        K[X, X] = prob["Qx"][t]
        K[X, W] = Qxw[t]
        K[X, L] = -I
        K[X, Ln] = A.T
        r[X] = -lx[t]
        # w_t row
        K[W, X] = Qxw[t].T
        K[W, W] = prob["Qw"][t]
        K[W, Ln] = B.T
        r[W] = -lw[t]
        # lam_{t+1} row
        K[Ln, X] = A
        K[Ln, W] = B
        K[Ln, Xn] = -I
        r[Ln] = -a[t]
    XN, LN = slice(xo[N], xo[N] + nx), slice(lo[N], lo[N] + nx)
    K[XN, XN] = prob["QxN"]
    K[XN, LN] = -I
    r[XN] = -lN
    return K, r


def split(z, nx, nu, N):
    """Unpack z into (x, w, lam) arrays."""
    lo, xo, wo, _ = _offsets(nx, nu, N)
    x = np.array([z[o:o + nx] for o in xo])
    lam = np.array([z[o:o + nx] for o in lo])
    w = np.array([z[o:o + nu] for o in wo]).reshape(N, nu)
    return x, w, lam


def pack(x, w, lam):
    N, nu = np.asarray(w).reshape(len(x) - 1, -1).shape
    parts = []
    for t in range(N + 1):
        parts.append(lam[t])
        parts.append(x[t])
        if t < N:
            parts.append(np.asarray(w[t]).reshape(-1))
    return np.concatenate(parts)


def solve_dense(prob):
    """Brute-force solution of P(N): LU solve of the dense KKT system."""
    nx, nu, N = dims(prob)
    K, r = assemble(prob)
    z = np.linalg.solve(K, r)
    x, w, lam = split(z, nx, nu, N)
    return dict(x=x, w=w, lam=lam)


def objective(prob, x, w):
    """Value of the objective of P(N) at (x, w), evaluated term by term."""
    nx, nu, N = dims(prob)
    Qxw = _get(prob, "Qxw", (N, nx, nu))
    lx, lw = _get(prob, "lx", (N, nx)), _get(prob, "lw", (N, nu))
    c = _get(prob, "c", (N,))
    lN = _get(prob, "lN", (nx,))
    J = 0.0
    for t in range(N):
        xt, wt = x[t], np.asarray(w[t]).reshape(-1)
        J += 0.5 * xt @ prob["Qx"][t] @ xt + xt @ Qxw[t] @ wt \
            + 0.5 * wt @ prob["Qw"][t] @ wt + lx[t] @ xt + lw[t] @ wt + c[t]
    J += 0.5 * x[N] @ prob["QxN"] @ x[N] + lN @ x[N] + float(prob.get("cN", 0.0))
    return J


def residual_blocks(prob, x, w, lam):
    """Blockwise residual rho = r - K z of the KKT system, computed without
    forming K.  Returns (rho_lam0 (nx,), rho_x (N+1,nx), rho_w (N,nu),
    rho_lam (N,nx) for the dynamics rows lam_1..lam_N)."""
    nx, nu, N = dims(prob)
    x, w, lam = (np.asarray(v, dtype=np.float64) for v in (x, w, lam))
    w = w.reshape(N, nu)
    Qxw = _get(prob, "Qxw", (N, nx, nu))
    a, lx = _get(prob, "a", (N, nx)), _get(prob, "lx", (N, nx))
    lw, lN = _get(prob, "lw", (N, nu)), _get(prob, "lN", (nx,))
    A, B, Qx, Qw = prob["A"], prob["B"], prob["Qx"], prob["Qw"]
    r_l0 = -np.asarray(prob["x0"]) + x[0]
    r_x = np.zeros((N + 1, nx))
    if N > 0:
        r_x[:N] = -lx - (np.einsum("tij,tj->ti", Qx, x[:N])
                         + np.einsum("tij,tj->ti", Qxw, w) - lam[:N]
                         + np.einsum("tji,tj->ti", A, lam[1:]))
    r_x[N] = -lN - (prob["QxN"] @ x[N] - lam[N])
    r_w = -lw - (np.einsum("tji,tj->ti", Qxw, x[:N]) + np.einsum("tij,tj->ti", Qw, w)
                 + np.einsum("tji,tj->ti", B, lam[1:]))
    r_l = -a - (np.einsum("tij,tj->ti", A, x[:N]) + np.einsum("tij,tj->ti", B, w) - x[1:])
    return r_l0, r_x, r_w, r_l


def rhs_norm_inf(prob):
    nx, nu, N = dims(prob)
    parts = [np.abs(np.asarray(prob["x0"])).max()]
    for key, shape in (("a", (N, nx)), ("lx", (N, nx)), ("lw", (N, nu)), ("lN", (nx,))):
        v = _get(prob, key, shape)
        if v.size:
            parts.append(np.abs(v).max())
    return max(parts)


def rel_residual(prob, x, w, lam):
    """||r - K z||_inf / ||r||_inf."""
    blocks = residual_blocks(prob, x, w, lam)
    num = max(np.abs(b).max() if b.size else 0.0 for b in blocks)
    return num / rhs_norm_inf(prob)


def rel_error(sol, ref):
    """max over the blocks x, w, lam of ||sol - ref||_inf / ||ref||_inf."""
    err = 0.0
    for key in ("x", "w", "lam"):
        r = np.asarray(ref[key], dtype=np.float64)
        if r.size == 0:
            continue
        d = np.abs(np.asarray(sol[key], dtype=np.float64).reshape(r.shape) - r).max()
        scale = np.abs(r).max()
        err = max(err, d / scale if scale > 0 else d)
    return err
