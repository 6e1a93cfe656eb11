"""Seeded synthetic UFTOC workloads.

This module only draws random problem data; it holds none of the solver's
arithmetic and is shared by the GPU path's callers and by the oracle's tests.

A problem is a dict of float64 arrays with row-major blocks:

    Qx (N,nx,nx)  Qw (N,nu,nu)  Qxw (N,nx,nu)  A (N,nx,nx)  B (N,nx,nu)
    a (N,nx)  lx (N,nx)  lw (N,nu)  c (N,)  QxN (nx,nx)  lN (nx,)  cN ()
    x0 (nx,)

Generators (the paper does not publish its test systems; these stand in for
them with the problem structure of Sec. 2):

* ``g1`` - time-invariant A with N(0,1) entries rescaled to spectral radius
  0.95 (materialised per stage), B ~ N(0,1), diagonal Qx, Qw with U[0.5,2]
  entries, Qxw = 0, a, lx, lw ~ N(0,1), c = 0, x0 ~ N(0,I).
* ``g2`` - time-varying A_t = A + 0.05 N(0,1) (A as in g1), B_t = N(0,1)/sqrt(nx),
  Qx_t = M M' + 0.1 I with fresh M ~ N(0,1), Qw diagonal U[0.5,2] and a cross
  term Qxw_t = beta_t 0.1 N(0,1) with beta_t = min(1, 0.5/||L^{-1} S R^{-1/2}||_F)
  (Qx = L L'), which keeps R - S' Qx^{-1} S >= 0.75 R, i.e. the stage Hessian
  positive definite.

The terminal cost is drawn like a stage Qx (reading: the configurations do not
state it) and lN ~ N(0,I).  Seeds are 151003110 + 1000*config + instance.
"""
import math

import numpy as np

SEED_BASE = 151003110


def seed_for(config, instance=0):
    return SEED_BASE + 1000 * int(config) + int(instance)


def _spectral_scale(A, rho=0.95):
    r = np.max(np.abs(np.linalg.eigvals(A)))
    return A * (rho / r)


def g1(nx, nu, N, seed):
    rng = np.random.default_rng(seed)
    A = _spectral_scale(rng.standard_normal((nx, nx)))
    B = rng.standard_normal((nx, nu))
    p = dict(
        Qx=np.stack([np.diag(rng.uniform(0.5, 2.0, nx)) for _ in range(N)]).reshape(N, nx, nx),
        Qw=np.stack([np.diag(rng.uniform(0.5, 2.0, nu)) for _ in range(N)]).reshape(N, nu, nu),
        Qxw=np.zeros((N, nx, nu)),
        A=np.broadcast_to(A, (N, nx, nx)).copy(),
        B=np.broadcast_to(B, (N, nx, nu)).copy(),
        a=rng.standard_normal((N, nx)),
        lx=rng.standard_normal((N, nx)),
        lw=rng.standard_normal((N, nu)),
        c=np.zeros(N),
        QxN=np.diag(rng.uniform(0.5, 2.0, nx)),
        lN=rng.standard_normal(nx),
        cN=np.float64(0.0),
        x0=rng.standard_normal(nx),
    )
    return p


def g1_invariant(nx, nu, N, seed):
    """G1 instance with the time-invariant A and B given once (stage axis of
    length 1, passed with stage stride 0) and the diagonal weights drawn in
    one call each.  Same distributions as ``g1``; a different random stream.
    For large batches of long horizons."""
    rng = np.random.default_rng(seed)
    A = _spectral_scale(rng.standard_normal((nx, nx)))
    B = rng.standard_normal((nx, nu))
    qx = rng.uniform(0.5, 2.0, (N, nx))
    qw = rng.uniform(0.5, 2.0, (N, nu))
    Qx = np.zeros((N, nx, nx))
    Qx[:, np.arange(nx), np.arange(nx)] = qx
    Qw = np.zeros((N, nu, nu))
    Qw[:, np.arange(nu), np.arange(nu)] = qw
    return dict(Qx=Qx, Qw=Qw, Qxw=np.zeros((1, nx, nu)), A=A[None].copy(), B=B[None].copy(),
                a=rng.standard_normal((N, nx)), lx=rng.standard_normal((N, nx)),
                lw=rng.standard_normal((N, nu)), c=np.zeros(N),
                QxN=np.diag(rng.uniform(0.5, 2.0, nx)), lN=rng.standard_normal(nx), cN=np.float64(0.0),
                x0=rng.standard_normal(nx))


def materialize(prob):
    """Copy of ``prob`` with every stage-axis-1 matrix repeated over the N
    stages (the form the oracle takes)."""
    N = prob["lx"].shape[0]
    q = dict(prob)
    for k in ("Qx", "Qw", "Qxw", "A", "B"):
        if k in q and q[k] is not None and q[k].shape[0] == 1 and N > 1:
            q[k] = np.repeat(q[k], N, axis=0)
    return q


def _cross_term(rng, Qx, Rdiag, nu):
    nx = Qx.shape[0]
    S = 0.1 * rng.standard_normal((nx, nu))
    L = np.linalg.cholesky(Qx)
    T = np.linalg.solve(L, S) / np.sqrt(Rdiag)[None, :]
    fro = np.linalg.norm(T)
    beta = 1.0 if fro == 0 else min(1.0, 0.5 / fro)
    return beta * S


def g2(nx, nu, N, seed, cross=True):
    rng = np.random.default_rng(seed)
    A0 = _spectral_scale(rng.standard_normal((nx, nx)))
    A = A0[None] + 0.05 * rng.standard_normal((N, nx, nx))
    B = rng.standard_normal((N, nx, nu)) / math.sqrt(nx)
    M = rng.standard_normal((N, nx, nx))
    Qx = M @ np.swapaxes(M, 1, 2) + 0.1 * np.eye(nx)[None]
    Rd = rng.uniform(0.5, 2.0, (N, nu))
    Qw = np.zeros((N, nu, nu))
    idx = np.arange(nu)
    Qw[:, idx, idx] = Rd
    if cross:
        Qxw = np.stack([_cross_term(rng, Qx[t], Rd[t], nu) for t in range(N)]).reshape(N, nx, nu)
    else:
        Qxw = np.zeros((N, nx, nu))
    MN = rng.standard_normal((nx, nx))
    p = dict(
        Qx=Qx, Qw=Qw, Qxw=Qxw, A=A, B=B,
        a=rng.standard_normal((N, nx)),
        lx=rng.standard_normal((N, nx)),
        lw=rng.standard_normal((N, nu)),
        c=np.zeros(N),
        QxN=MN @ MN.T + 0.1 * np.eye(nx),
        lN=rng.standard_normal(nx),
        cN=np.float64(0.0),
        x0=rng.standard_normal(nx),
    )
    return p


def with_costs(prob, seed):
    """Copy of ``prob`` with c_t, cN ~ N(0,1) (for objective-value checks)."""
    rng = np.random.default_rng(seed)
    q = dict(prob)
    q["c"] = rng.standard_normal(prob["Qx"].shape[0])
    q["cN"] = np.float64(rng.standard_normal())
    return q


# ---------------------------------------------------------------- device side
def g2_torch(nx, nu, N, count, seed, device="cuda", cross=True):
    """Batch of ``count`` g2-distributed instances drawn directly in device
    memory with torch's generator (for batches too large to draw on the host).
    Same distributions as ``g2``; a different random stream.  Returns a dict
    of stacked tensors with a leading instance axis."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    # spectral scaling of the base A per instance (host eigvals, tiny)
    A0 = torch.randn((count, nx, nx), generator=gen, **f64)
    rad = torch.linalg.eigvals(A0.cpu()).abs().amax(dim=-1).to(device)
    A0 = A0 * (0.95 / rad)[:, None, None]
    A = A0[:, None] + 0.05 * torch.randn((count, N, nx, nx), generator=gen, **f64)
    B = torch.randn((count, N, nx, nu), generator=gen, **f64) / math.sqrt(nx)
    Qx = torch.empty((count, N, nx, nx), **f64)
    eye = torch.eye(nx, **f64)
    for i in range(count):          # chunked so the temporaries stay small
        M = torch.randn((N, nx, nx), generator=gen, **f64)
        Qx[i] = torch.matmul(M, M.transpose(1, 2).contiguous()) + 0.1 * eye
    Rd = torch.rand((count, N, nu), generator=gen, **f64) * 1.5 + 0.5
    Qw = torch.diag_embed(Rd)
    if cross:
        Qxw = torch.empty((count, N, nx, nu), **f64)
        for i in range(count):
            S = 0.1 * torch.randn((N, nx, nu), generator=gen, **f64)
            L = torch.linalg.cholesky(Qx[i])
            T = torch.linalg.solve_triangular(L, S, upper=False) / Rd[i].sqrt()[:, None, :]
            fro = torch.linalg.matrix_norm(T)
            beta = torch.clamp(0.5 / fro, max=1.0)
            Qxw[i] = beta[:, None, None] * S
    else:
        Qxw = torch.zeros((count, N, nx, nu), **f64)
    MN = torch.randn((count, nx, nx), generator=gen, **f64)
    QxN = torch.matmul(MN, MN.transpose(1, 2).contiguous()) + 0.1 * eye
    return dict(
        Qx=Qx, Qw=Qw, Qxw=Qxw, A=A, B=B,
        a=torch.randn((count, N, nx), generator=gen, **f64),
        lx=torch.randn((count, N, nx), generator=gen, **f64),
        lw=torch.randn((count, N, nu), generator=gen, **f64),
        c=torch.zeros((count, N), **f64),
        QxN=QxN,
        lN=torch.randn((count, nx), generator=gen, **f64),
        cN=torch.zeros((count,), **f64),
        x0=torch.randn((count, nx), generator=gen, **f64),
    )


def c5_torch(nx, nu, N, count, seed, device="cuda"):
    """Batch of the large-block configuration's instances drawn in device
    memory: time-varying dynamics A_t = A + 0.05 N(0,1) (A scaled to spectral
    radius 0.95, the G2 rule), and the G1 rest, time-invariant per instance
    and given once (stage axis of length 1, passed with stage stride 0):
    B ~ N(0,1), Q_x = diag U[0.5, 2], Q_w = diag U[0.5, 2], no cross term,
    Q_{x,N} = diag U[0.5, 2]; a_t, l_{x,t}, l_{w,t}, l_N, xbar_0 ~ N(0,1),
    c_t = 0.  Only A_t and the stage vectors grow with N (about 131 KB of
    FP64 per stage at n_x = 128), so a batch of 64 at N = 16384 fits in HBM."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    A0 = torch.randn((count, nx, nx), generator=gen, **f64)
    rad = torch.linalg.eigvals(A0.cpu()).abs().amax(dim=-1).to(device)
    A0 = A0 * (0.95 / rad)[:, None, None]
    A = torch.empty((count, N, nx, nx), **f64)
    for i in range(count):          # chunked so the temporaries stay small
        A[i] = A0[i][None] + 0.05 * torch.randn((N, nx, nx), generator=gen, **f64)
    B = torch.randn((count, 1, nx, nu), generator=gen, **f64)
    Qx = torch.diag_embed(torch.rand((count, 1, nx), generator=gen, **f64) * 1.5 + 0.5)
    Qw = torch.diag_embed(torch.rand((count, 1, nu), generator=gen, **f64) * 1.5 + 0.5)
    QxN = torch.diag_embed(torch.rand((count, nx), generator=gen, **f64) * 1.5 + 0.5)
    return dict(
        Qx=Qx, Qw=Qw, A=A, B=B,
        a=torch.randn((count, N, nx), generator=gen, **f64),
        lx=torch.randn((count, N, nx), generator=gen, **f64),
        lw=torch.randn((count, N, nu), generator=gen, **f64),
        c=torch.zeros((count, N), **f64),
        QxN=QxN,
        lN=torch.randn((count, nx), generator=gen, **f64),
        cN=torch.zeros((count,), **f64),
        x0=torch.randn((count, nx), generator=gen, **f64),
    )


def g1_invariant_torch(nx, nu, horizons, seed, device="cuda"):
    """Batch of G1 instances with the given horizons drawn in device memory:
    A scaled to spectral radius 0.95 and B ~ N(0,1), both time-invariant and
    given once (stage axis of length 1); Q_x, Q_w diagonal U[0.5, 2] per
    stage; no cross term; a_t, l_{x,t}, l_{w,t}, l_N, xbar_0 ~ N(0,1); c_t = 0;
    Q_{x,N} = diag U[0.5, 2].  Same distributions as ``g1_invariant``, a
    different random stream.  Returns a dict of per-instance tensor lists
    (views into a few large tensors)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    Ns = [int(n) for n in horizons]
    cnt, S = len(Ns), int(sum(Ns))
    A0 = torch.randn((cnt, nx, nx), generator=gen, **f64)
    rad = torch.linalg.eigvals(A0.cpu()).abs().amax(dim=-1).to(device)
    A = (A0 * (0.95 / rad)[:, None, None])[:, None]
    B = torch.randn((cnt, 1, nx, nu), generator=gen, **f64)
    Qx = torch.diag_embed(torch.rand((S, nx), generator=gen, **f64) * 1.5 + 0.5)
    Qw = torch.diag_embed(torch.rand((S, nu), generator=gen, **f64) * 1.5 + 0.5)
    a = torch.randn((S, nx), generator=gen, **f64)
    lx = torch.randn((S, nx), generator=gen, **f64)
    lw = torch.randn((S, nu), generator=gen, **f64)
    c = torch.zeros((S,), **f64)
    QxN = torch.diag_embed(torch.rand((cnt, nx), generator=gen, **f64) * 1.5 + 0.5)
    lN = torch.randn((cnt, nx), generator=gen, **f64)
    x0 = torch.randn((cnt, nx), generator=gen, **f64)
    out = {k: list(torch.split(v, Ns)) for k, v in (("Qx", Qx), ("Qw", Qw), ("a", a), ("lx", lx), ("lw", lw),
                                                      ("c", c))}
    out.update(A=list(A), B=list(B), QxN=list(QxN), lN=list(lN), x0=list(x0),
               cN=list(torch.zeros((cnt,), **f64)))
    return out


def instance_to_numpy(batch, i):
    """Instance ``i`` of a stacked torch batch as a numpy problem dict."""
    out = {}
    for k, v in batch.items():
        out[k] = v[i].detach().cpu().numpy().astype(np.float64)
    out["cN"] = np.float64(out["cN"])
    return out


def mhe_problem(nx, ny, Nm, seed, correlated=False, nw=None):
    """Seeded linear-Gaussian MHE problem with samples k = 0..Nm and process
    noise of dimension nw (default n_x): A_k = A + 0.05 N(0,1) (A scaled to
    spectral radius 0.95), B_k (n_x x n_w), C_k N(0,1) (B_k / sqrt(nx)),
    small affine and nominal terms, measurements N(0,1), covariances
    M M'/k + 0.5 I and, if `correlated`, a cross covariance
    0.2 N(0,1) / sqrt(max(nw, ny)) (small enough for the joint covariance to
    stay positive definite).  Returns a dict of numpy arrays with a leading sample axis."""
    nw = nx if nw is None else nw
    rng = np.random.default_rng(seed)
    A0 = _spectral_scale(rng.standard_normal((nx, nx)))

    def spd(k, n):
        M = rng.standard_normal((n, k, k))
        return M @ np.swapaxes(M, 1, 2) / k + 0.5 * np.eye(k)[None]

    K = Nm + 1
    p = dict(
        A=A0[None] + 0.05 * rng.standard_normal((K, nx, nx)),
        B=rng.standard_normal((K, nx, nw)) / math.sqrt(nx),
        a=0.1 * rng.standard_normal((K, nx)),
        C=rng.standard_normal((K, ny, nx)),
        d=0.1 * rng.standard_normal((K, ny)),
        y=rng.standard_normal((K, ny)),
        wtil=0.1 * rng.standard_normal((K, nw)),
        vtil=0.1 * rng.standard_normal((K, ny)),
        Qw=spd(nw, K),
        Qv=spd(ny, K),
        xtil0=rng.standard_normal(nx),
        Ptil0=spd(nx, 1)[0],
    )
    p["Qwv"] = 0.2 * rng.standard_normal((K, nw, ny)) / math.sqrt(max(nw, ny)) if correlated else None
    return p
