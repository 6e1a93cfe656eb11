"""The KKT system of P(N) solved in exact rational arithmetic.

Test infrastructure only (see the package docstring).

For tiny problems with rational data the KKT system (assembled exactly as in
``oracle.kkt``, rows from the Lagrangian of P(N), Sec. 2-3) is solved by
Gauss-Jordan elimination over ``fractions.Fraction``.  The result is exact, so
it pins the floating-point oracle without any rounding or tolerance argument
of its own.
"""
from fractions import Fraction


def _F(v):
    return v if isinstance(v, Fraction) else Fraction(v)


def assemble(prob):
    """Exact KKT matrix and right-hand side.  ``prob`` holds nested lists of
    Fractions (or ints) with the shapes of the float oracle's dict."""
    N, nx, nu = len(prob["Qx"]), len(prob["QxN"]), len(prob["Qw"][0]) if prob["Qw"] else 0
    stride = 2 * nx + nu
    size = N * stride + 2 * nx
    lo = [t * stride for t in range(N + 1)]
    xo = [t * stride + nx for t in range(N + 1)]
    wo = [t * stride + 2 * nx for t in range(N)]
    K = [[Fraction(0)] * size for _ in range(size)]
    r = [Fraction(0)] * size
    for i in range(nx):
        K[lo[0] + i][xo[0] + i] = Fraction(-1)
        r[lo[0] + i] = -_F(prob["x0"][i])
    for t in range(N):
        for i in range(nx):
            row = xo[t] + i
            for j in range(nx):
                K[row][xo[t] + j] = _F(prob["Qx"][t][i][j])
                K[row][lo[t + 1] + j] = _F(prob["A"][t][j][i])
            for j in range(nu):
                K[row][wo[t] + j] = _F(prob["Qxw"][t][i][j])
            K[row][lo[t] + i] = Fraction(-1)
            r[row] = -_F(prob["lx"][t][i])
        for i in range(nu):
            row = wo[t] + i
            for j in range(nx):
                K[row][xo[t] + j] = _F(prob["Qxw"][t][j][i])
                K[row][lo[t + 1] + j] = _F(prob["B"][t][j][i])
            for j in range(nu):
                K[row][wo[t] + j] = _F(prob["Qw"][t][i][j])
            r[row] = -_F(prob["lw"][t][i])
        for i in range(nx):
            row = lo[t + 1] + i
            for j in range(nx):
                K[row][xo[t] + j] = _F(prob["A"][t][i][j])
            for j in range(nu):
                K[row][wo[t] + j] = _F(prob["B"][t][i][j])
            K[row][xo[t + 1] + i] = Fraction(-1)
            r[row] = -_F(prob["a"][t][i])
    for i in range(nx):
        row = xo[N] + i
        for j in range(nx):
            K[row][xo[N] + j] = _F(prob["QxN"][i][j])
        K[row][lo[N] + i] = Fraction(-1)
        r[row] = -_F(prob["lN"][i])
    return K, r, (lo, xo, wo)


def gauss_jordan(K, r):
    """Solve K z = r exactly (partial pivoting on the first nonzero)."""
    n = len(r)
    M = [row[:] + [r[i]] for i, row in enumerate(K)]
    for col in range(n):
        piv = next(i for i in range(col, n) if M[i][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [v / p for v in M[col]]
        for i in range(n):
            if i != col and M[i][col] != 0:
                f = M[i][col]
                M[i] = [vi - f * vc for vi, vc in zip(M[i], M[col])]
    return [M[i][n] for i in range(n)]


def solve(prob):
    """Exact (x, w, lam) and optimal value of P(N) for rational data."""
    K, r, (lo, xo, wo) = assemble(prob)
    z = gauss_jordan(K, r)
    N, nx = len(prob["Qx"]), len(prob["QxN"])
    nu = len(prob["Qw"][0]) if N else 0
    x = [[z[o + i] for i in range(nx)] for o in xo]
    lam = [[z[o + i] for i in range(nx)] for o in lo]
    w = [[z[o + i] for i in range(nu)] for o in wo]
    # objective, term by term
    J = Fraction(0)
    for t in range(N):
        xt, wt = x[t], w[t]
        for i in range(nx):
            for j in range(nx):
                J += Fraction(1, 2) * xt[i] * _F(prob["Qx"][t][i][j]) * xt[j]
            for j in range(nu):
                J += xt[i] * _F(prob["Qxw"][t][i][j]) * wt[j]
            J += _F(prob["lx"][t][i]) * xt[i]
        for i in range(nu):
            for j in range(nu):
                J += Fraction(1, 2) * wt[i] * _F(prob["Qw"][t][i][j]) * wt[j]
            J += _F(prob["lw"][t][i]) * wt[i]
        J += _F(prob["c"][t])
    for i in range(nx):
        for j in range(nx):
            J += Fraction(1, 2) * x[N][i] * _F(prob["QxN"][i][j]) * x[N][j]
        J += _F(prob["lN"][i]) * x[N][i]
    J += _F(prob["cN"])
    return dict(x=x, w=w, lam=lam, obj=J)
