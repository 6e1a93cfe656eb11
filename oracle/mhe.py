"""MHE problem (Sec. 2, eq. "org_mhe") to UFTOC conversion, and the RTS
smoother for the linear-Gaussian case.

Test infrastructure only (see the package docstring).

Conversion (Sec. 2): a state x_{-1} = xtil_0 and a noise w_{-1} = x_0 - xtil_0
are prepended, time is shifted by t = k + 1 and N = N_mhe + 2.  Stage 0 has
Qx = 0, Qxw = 0, Qw = Ptil_0^{-1}, A = I, B = I, a = 0; the terminal cost is
zero.  Stage t >= 1 carries the MHE data of sample k = t - 1.

With [[W, S], [S', V]] the inverse of the joint noise covariance (W is
n_w x n_w, S is n_w x n_y) and ytil = y - d - vtil, expanding the stage cost
in (x, w) gives

    Qx = C' V C,  Qxw = -C' S',  Qw = W,
    lx = C' (S' wtil - V ytil),  lw = S ytil - W wtil,
    c  = 1/2 wtil' W wtil - wtil' S ytil + 1/2 ytil' V ytil.

The printed formulas place S without these transposes, which is dimensionally
consistent only if S is read as n_y x n_w; the expressions above are the ones
derived from the cost and coincide with the printed ones when S = 0.

The UFTOC noise dimension is n_x at stage 0 and n_w afterwards, while P(N)
has one input dimension n_u for all stages.  Reading: every stage's input
is padded to n_u = max(n_x, n_w) with inputs that act on nothing (zero
columns of B and Q_xw, an identity block of Q_w, zero l_w).  They are
decoupled from the rest and strictly convex, so they are zero at the
optimum and the other unknowns are those of the unpadded problem.
"""
import numpy as np


def mhe_to_uftoc(A, B, a, C, d, y, xtil0, Ptil0, wtil, vtil, Qw_cov, Qv_cov, Qwv_cov=None):
    """Arrays indexed by the MHE sample k = 0..Nmhe.  Returns a UFTOC dict."""
    Nm = len(A) - 1
    nx, nw = A[0].shape[0], B[0].shape[1]
    nu = max(nx, nw)
    N = Nm + 2

    def cols(M, n):          # M (rows x n) followed by zero columns up to nu
        out = np.zeros((M.shape[0], nu))
        out[:, :n] = M
        return out

    def weight(M, n):        # blockdiag(M, I) of size nu
        out = np.eye(nu)
        out[:n, :n] = M
        return out

    def vec(v, n):
        out = np.zeros(nu)
        out[:n] = v
        return out

    prob = {k: [] for k in ("Qx", "Qw", "Qxw", "A", "B", "a", "lx", "lw", "c")}
    # stage 0: arrival cost as noise cost on w_{-1}
    prob["Qx"].append(np.zeros((nx, nx)))
    prob["Qw"].append(weight(np.linalg.inv(Ptil0), nx))
    prob["Qxw"].append(np.zeros((nx, nu)))
    prob["A"].append(np.eye(nx))
    prob["B"].append(cols(np.eye(nx), nx))
    prob["a"].append(np.zeros(nx))
    prob["lx"].append(np.zeros(nx))
    prob["lw"].append(np.zeros(nu))
    prob["c"].append(0.0)
    for k in range(Nm + 1):
        ny = C[k].shape[0]
        cov = np.zeros((nw + ny, nw + ny))
        cov[:nw, :nw] = Qw_cov[k]
        cov[nw:, nw:] = Qv_cov[k]
        if Qwv_cov is not None:
            cov[:nw, nw:] = Qwv_cov[k]
            cov[nw:, :nw] = Qwv_cov[k].T
        inv = np.linalg.inv(cov)
        W, S, V = inv[:nw, :nw], inv[:nw, nw:], inv[nw:, nw:]
        yt = y[k] - d[k] - vtil[k]
        Ck = C[k]
        prob["Qx"].append(Ck.T @ V @ Ck)
        prob["Qxw"].append(cols(-Ck.T @ S.T, nw))
        prob["Qw"].append(weight(W, nw))
        prob["lx"].append(Ck.T @ (S.T @ wtil[k] - V @ yt))
        prob["lw"].append(vec(S @ yt - W @ wtil[k], nw))
        prob["c"].append(0.5 * wtil[k] @ W @ wtil[k] - wtil[k] @ S @ yt + 0.5 * yt @ V @ yt)
        prob["A"].append(A[k])
        prob["B"].append(cols(B[k], nw))
        prob["a"].append(a[k])
    out = {k: np.array(v) for k, v in prob.items()}
    out["QxN"] = np.zeros((nx, nx))
    out["lN"] = np.zeros(nx)
    out["cN"] = 0.0
    out["x0"] = np.asarray(xtil0, dtype=np.float64)
    assert out["Qx"].shape[0] == N
    return out


def rts_smoother(A, B, a, C, d, y, xtil0, Ptil0, wtil, vtil, Qw_cov, Qv_cov):
    """Kalman filter plus Rauch-Tung-Striebel smoother for
    x_{k+1} = A x + B w + a, y = C x + v + d, w ~ N(wtil, Qw), v ~ N(vtil, Qv),
    x_0 ~ N(xtil0, Ptil0), independent noises.  Returns the smoothed means of
    x_0..x_{Nmhe+1} (the last one is the prediction past the final sample)."""
    Nm = len(A) - 1
    m_pred, P_pred = np.asarray(xtil0, dtype=np.float64), np.asarray(Ptil0, dtype=np.float64)
    mf, Pf, mp, Pp = [], [], [m_pred], [P_pred]
    for k in range(Nm + 1):
        Ck = C[k]
        e = (y[k] - d[k] - vtil[k]) - Ck @ m_pred
        Sk = Ck @ P_pred @ Ck.T + Qv_cov[k]
        Kk = np.linalg.solve(Sk, Ck @ P_pred).T
        m_f = m_pred + Kk @ e
        P_f = P_pred - Kk @ Ck @ P_pred
        mf.append(m_f)
        Pf.append(P_f)
        m_pred = A[k] @ m_f + B[k] @ wtil[k] + a[k]
        P_pred = A[k] @ P_f @ A[k].T + B[k] @ Qw_cov[k] @ B[k].T
        mp.append(m_pred)
        Pp.append(P_pred)
    ms = [None] * (Nm + 2)
    ms[Nm + 1] = mp[Nm + 1]
    for k in range(Nm, -1, -1):
        J = np.linalg.solve(Pp[k + 1], A[k] @ Pf[k]).T
        ms[k] = mf[k] + J @ (ms[k + 1] - mp[k + 1])
    return np.array(ms)
