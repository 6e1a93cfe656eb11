"""Closed-form reduced subproblem (Theorem 1) and master problem (Sec. 4.3).

Test infrastructure only (see the package docstring).

A subinterval of P(N) (Sec. 4.1, eq. "sub_problem_dscr") is reduced with the
preliminary choice Phat = 0, Psihat = 0, chat = 0 (Sec. 4.2).  The preliminary
solution is the serial Riccati oracle (Alg. 1-2) run on the subinterval with a
zero terminal.  From it the reduced quantities are written out with the
paper's definitions, *not* with the recursion of Alg. 4:

    Qx_hat = P_{0,0},  lx_hat = -Psi_{0,0},  c_hat = cbar_{0,0}     (eq. Qxh_lxh_def)
    A_hat  = prod_{t=0}^{N-1} (A_t + B_t K_{0,t+1})                (eq. QuA)
    S      = [ prod_{t=tau+1}^{N-1}(A_t + B_t K_{0,t+1}) B_tau ]_tau (eq. B)
    a_hat  = sum_tau prod_{t=tau+1}^{N-1}(...) (a_tau + B_tau k_{0,tau+1}) (eq. a)
    Qbar   = blockdiag(G_{0,1}, ..., G_{0,N})                        (eq. QuA)
    Qw_hat = B_hat = S Qbar^{-1} S'                                  (eq. Qh_Bh_alternative_def)

Products follow the paper's convention (Sec. 1): the factor with the larger
index stands on the left.  Reading of the elided middle columns of S: column
block tau is the product over t = tau+1..N-1 times B_tau.

The last subinterval, whose terminal cost is known, is eliminated entirely
(Sec. 4.2, last paragraph): its reduced form is the terminal cost
(P_0, -Psi_0, cbar_0) of a Riccati pass with the true terminal.

The rank-revealing form (Sec. 4.2, eqs. Bh_def and Gh_Hh_def) takes an
orthonormal basis U_1 of range(S') with n_uo = rank(S') <= n_x columns:
    Qw_hat = U_1' Qbar^{-1} U_1  (n_uo x n_uo, positive definite),
    B_hat  = S Qbar^{-1} U_1     (n_x x n_uo),
so that the master stage has n_uo inputs and its G_hat is nonsingular even
when S' is rank deficient (N_s n_u < n_x, or a subinterval whose inputs do
not reach every state direction).  U_1 comes from the singular value
decomposition of S' with numpy's rank rule (singular values above
max(dims) eps sigma_max).  Master problems whose stages have different input
dimensions are solved here from their KKT system written out densely.
"""
import numpy as np

from . import riccati


def sub_problem(prob, t0, t1, terminal=None):
    """Stages t0..t1-1 of ``prob`` as a UFTOC problem (eq. sub_problem_dscr).
    ``terminal`` = (P, Psi, cbar) of the cost to go at t1; None gives the
    preliminary choice 0."""
    nx = prob["QxN"].shape[0]
    sub = {}
    for key in ("Qx", "Qw", "Qxw", "A", "B", "a", "lx", "lw", "c"):
        if prob.get(key) is not None:
            sub[key] = np.ascontiguousarray(prob[key][t0:t1])
    if terminal is None:
        sub["QxN"], sub["lN"], sub["cN"] = np.zeros((nx, nx)), np.zeros(nx), 0.0
    else:
        P, Psi, cb = terminal
        sub["QxN"], sub["lN"], sub["cN"] = np.asarray(P), -np.asarray(Psi), float(cb)
    sub["x0"] = np.zeros(nx)
    return sub


def reduce_closed_form(sub):
    """Reduced form of a subproblem with unknown terminal (Theorem 1 with the
    T-transform).  Returns dict(A, B, a, Qx, Qw, lx, c)."""
    nx = sub["QxN"].shape[0]
    N = sub["Qx"].shape[0]
    pre = riccati.solve(sub, want_factors=True)          # preliminary P=0 solve
    K, k, G = pre["K"], pre["k"], pre["G"]
    a = sub.get("a")
    a = np.zeros((N, nx)) if a is None else a
    Acl = [sub["A"][t] + sub["B"][t] @ K[t] for t in range(N)]

    def prod(lo, hi):                                     # prod_{t=lo}^{hi} Acl_t
        M = np.eye(nx)
        for t in range(lo, hi + 1):
            M = Acl[t] @ M                                # later index on the left
        return M

    A_hat = prod(0, N - 1)
    S = np.concatenate([prod(tau + 1, N - 1) @ sub["B"][tau] for tau in range(N)], axis=1)
    a_hat = sum(prod(tau + 1, N - 1) @ (a[tau] + sub["B"][tau] @ k[tau]) for tau in range(N))
    nu = sub["Qw"].shape[1]
    Qbar = np.zeros((N * nu, N * nu))
    for t in range(N):
        Qbar[t * nu:(t + 1) * nu, t * nu:(t + 1) * nu] = G[t]
    Qw_hat = S @ np.linalg.solve(Qbar, S.T)
    return dict(A=A_hat, B=Qw_hat, a=a_hat, Qx=pre["P"][0], Qw=Qw_hat,
                lx=-pre["Psi"][0], c=pre["cbar"][0], S=S, Qbar=Qbar)


def eliminate_last(sub):
    """Full elimination of the last subinterval (known terminal): returns the
    terminal cost (QxN, lN, cN) it contributes to the master problem."""
    pre = riccati.solve(sub, want_factors=True)
    return pre["P"][0], -pre["Psi"][0], pre["cbar"][0]


def master_problem(prob, bounds):
    """Master problem (eq. red_mpc_problem) of P(N) for the batch boundaries
    ``bounds`` = [t_0=0, t_1, ..., t_{p+1}=N].  Stage i is the reduced form of
    batch i < p; the last batch gives the terminal cost."""
    nx = prob["QxN"].shape[0]
    p = len(bounds) - 2
    stages = [reduce_closed_form(sub_problem(prob, bounds[i], bounds[i + 1]))
              for i in range(p)]
    last = sub_problem(prob, bounds[p], bounds[p + 1],
                       terminal=(prob["QxN"], -np.asarray(prob.get("lN", np.zeros(nx))),
                                 float(prob.get("cN", 0.0))))
    QxN, lN, cN = eliminate_last(last)
    m = dict(
        Qx=np.array([s["Qx"] for s in stages]).reshape(p, nx, nx),
        Qw=np.array([s["Qw"] for s in stages]).reshape(p, nx, nx),
        Qxw=np.zeros((p, nx, nx)),
        A=np.array([s["A"] for s in stages]).reshape(p, nx, nx),
        B=np.array([s["B"] for s in stages]).reshape(p, nx, nx),
        a=np.array([s["a"] for s in stages]).reshape(p, nx),
        lx=np.array([s["lx"] for s in stages]).reshape(p, nx),
        lw=np.zeros((p, nx)),
        c=np.array([s["c"] for s in stages]).reshape(p),
        QxN=QxN, lN=lN, cN=cN, x0=np.asarray(prob["x0"]))
    return m


def reduce_rank_revealing(sub):
    """Reduced form of a subproblem with the U_1 basis (eq. Bh_def).
    Returns dict(A, B (nx x nuo), a, Qx, Qw (nuo x nuo), lx, c, nuo)."""
    red = reduce_closed_form(sub)
    S, Qbar = red["S"], red["Qbar"]
    U, sv, _ = np.linalg.svd(S.T, full_matrices=False)
    tol = (sv[0] * max(S.shape) * np.finfo(float).eps) if sv.size else 0.0
    r = int(np.sum(sv > tol))
    U1 = U[:, :r]
    QinvU1 = np.linalg.solve(Qbar, U1)
    return dict(A=red["A"], B=S @ QinvU1, a=red["a"], Qx=red["Qx"], Qw=U1.T @ QinvU1,
                lx=red["lx"], c=red["c"], nuo=r)


def master_problem_rr(prob, bounds):
    """Master problem with rank-revealing stages: a list of per-stage dicts
    (A, B, a, Qx, Qw, lx, c, nuo) and the terminal (QxN, lN, cN), x0."""
    nx = prob["QxN"].shape[0]
    p = len(bounds) - 2
    stages = [reduce_rank_revealing(sub_problem(prob, bounds[i], bounds[i + 1])) for i in range(p)]
    last = sub_problem(prob, bounds[p], bounds[p + 1],
                       terminal=(prob["QxN"], -np.asarray(prob.get("lN", np.zeros(nx))),
                                 float(prob.get("cN", 0.0))))
    QxN, lN, cN = eliminate_last(last)
    return dict(stages=stages, QxN=QxN, lN=lN, cN=cN, x0=np.asarray(prob["x0"]))


def solve_master_dense(m):
    """Solve a master problem from master_problem_rr by its KKT system:
    minimise sum_i (1/2 x_i'Qx_i x_i + 1/2 w_i'Qw_i w_i + lx_i'x_i + c_i)
    + 1/2 x_p'QxN x_p + lN'x_p + cN subject to x_0 = x0 and
    x_{i+1} = A_i x_i + B_i w_i + a_i.  Returns x (p+1, nx), w (list),
    lam (p+1, nx) with the sign convention of P(N) (lam_i is the multiplier
    of the dynamics into x_i, lam_0 that of the initial condition) and obj."""
    st = m["stages"]
    p = len(st)
    nx = m["QxN"].shape[0]
    nus = [s["nuo"] for s in st]
    xo = [i * nx for i in range(p + 1)]
    wo, o = [], (p + 1) * nx
    for r in nus:
        wo.append(o)
        o += r
    nz, nc = o, (p + 1) * nx
    H = np.zeros((nz, nz))
    g = np.zeros(nz)
    const = float(m["cN"]) + sum(float(s["c"]) for s in st)
    C = np.zeros((nc, nz))
    b = np.zeros(nc)
    for i, s in enumerate(st):
        H[xo[i]:xo[i] + nx, xo[i]:xo[i] + nx] = s["Qx"]
        H[wo[i]:wo[i] + nus[i], wo[i]:wo[i] + nus[i]] = s["Qw"]
        g[xo[i]:xo[i] + nx] = s["lx"]
    H[xo[p]:xo[p] + nx, xo[p]:xo[p] + nx] = m["QxN"]
    g[xo[p]:xo[p] + nx] = m["lN"]
    # constraint rows: x_0 = x0; then x_{i+1} - A_i x_i - B_i w_i = a_i
    C[0:nx, 0:nx] = np.eye(nx)
    b[0:nx] = m["x0"]
    for i, s in enumerate(st):
        r = slice((i + 1) * nx, (i + 2) * nx)
        C[r, xo[i + 1]:xo[i + 1] + nx] = np.eye(nx)
        C[r, xo[i]:xo[i] + nx] = -s["A"]
        C[r, wo[i]:wo[i] + nus[i]] = -s["B"]
        b[r] = s["a"]
    K = np.block([[H, C.T], [C, np.zeros((nc, nc))]])
    sol = np.linalg.solve(K, np.concatenate([-g, b]))
    z, nu_ = sol[:nz], sol[nz:]
    x = np.array([z[xo[i]:xo[i] + nx] for i in range(p + 1)])
    w = [z[wo[i]:wo[i] + nus[i]] for i in range(p)]
    obj = 0.5 * z @ H @ z + g @ z + const
    # stationarity in x_i: Qx_i x_i + lx_i + nu_i - A_i' nu_{i+1} = 0; with
    # lam = -nu this is the x row of P(N): Qx x + lx - lam_i + A' lam_{i+1} = 0
    lam = -nu_.reshape(p + 1, nx)
    return dict(x=x, w=w, lam=lam, obj=float(obj))
