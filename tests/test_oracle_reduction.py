"""Pins of the closed-form reduction (Theorem 1, eqs. of Sec. 4.2) and of the
master problem (Sec. 4.3) against the full problem solved by brute force."""
import numpy as np
import pytest

from oracle import kkt, reduction, riccati
from paper_1510_03110_amd import workloads as W


def _terminal(rng, nx):
    M = rng.standard_normal((nx, nx))
    return M @ M.T + 0.5 * np.eye(nx), rng.standard_normal(nx), float(rng.standard_normal())


@pytest.mark.parametrize("nx,nu,Ns", [(3, 2, 4), (4, 2, 2), (2, 3, 3), (4, 4, 1)])
def test_theorem1_reduced_problem_equals_subproblem(nx, nu, Ns):
    """For an arbitrary terminal (Phat, Psihat, chat) and initial state, the
    one-stage reduced problem of Theorem 1 has the same optimal value and the
    same final state as the subproblem it replaces (eq. sub_problem_dscr)."""
    rng = np.random.default_rng(nx * 31 + Ns)
    prob = W.with_costs(W.g2(nx, nu, Ns, seed=nx + Ns), seed=2)
    red = reduction.reduce_closed_form(reduction.sub_problem(prob, 0, Ns))
    for trial in range(3):
        Ph, Psih, ch = _terminal(rng, nx)
        x0 = rng.standard_normal(nx)
        sub = reduction.sub_problem(prob, 0, Ns, terminal=(Ph, Psih, ch))
        sub["x0"] = x0
        full = riccati.solve(sub)
        one = dict(Qx=red["Qx"][None], Qw=red["Qw"][None], Qxw=np.zeros((1, nx, nx)),
                   A=red["A"][None], B=red["B"][None], a=red["a"][None],
                   lx=red["lx"][None], lw=np.zeros((1, nx)), c=np.array([red["c"]]),
                   QxN=Ph, lN=-Psih, cN=ch, x0=x0)
        # the reduced input cost may be singular when Ns*nu < nx; use LU then
        r1 = kkt.solve_dense(one) if Ns * nu < nx else riccati.solve(one)
        if "obj" not in r1:
            r1["obj"] = kkt.objective(one, r1["x"], r1["w"])
        np.testing.assert_allclose(r1["x"][1], full["x"][Ns], rtol=1e-9, atol=1e-9)
        assert abs(r1["obj"] - full["obj"]) <= 1e-9 * max(1.0, abs(full["obj"]))


def test_reduced_input_weight_is_gram_of_S():
    """Q_w_hat = S Qbar^{-1} S' is symmetric positive semidefinite, and
    positive definite when Ns*nu >= nx (generic data)."""
    prob = W.g2(4, 2, 3, seed=1)
    red = reduction.reduce_closed_form(reduction.sub_problem(prob, 0, 3))
    Q = red["Qw"]
    assert np.allclose(Q, Q.T)
    assert np.linalg.eigvalsh(Q).min() > 1e-8


@pytest.mark.parametrize("gen,nx,nu,N,bounds", [
    ("g2", 3, 2, 12, [0, 4, 8, 12]),
    ("g2", 4, 2, 13, [0, 3, 6, 9, 12, 13]),       # ragged last batch of length 1
    ("g1", 4, 2, 16, [0, 5, 10, 16]),
    ("g2", 2, 1, 9, [0, 2, 4, 6, 8, 9]),
])
def test_master_problem_equals_original(gen, nx, nu, N, bounds):
    """The master problem (eq. red_mpc_problem) built from the closed-form
    reductions has x_hat_i = x_{t_i}, cost to go P_hat, Psi_hat, c_hat equal to
    the serial values at t_i, and the same optimal value as P(N)."""
    prob = W.with_costs(getattr(W, gen)(nx, nu, N, seed=N * 7 + nx), seed=5)
    full = riccati.solve(prob, want_factors=True)
    dense = kkt.solve_dense(prob)
    assert kkt.rel_error(full, dense) < 1e-11
    m = reduction.master_problem(prob, bounds)
    ms = riccati.solve(m, want_factors=True)
    for i, t in enumerate(bounds[:-1]):
        np.testing.assert_allclose(ms["x"][i], full["x"][t], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(ms["P"][i], full["P"][t], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(ms["Psi"][i], full["Psi"][t], rtol=1e-9, atol=1e-9)
        assert abs(ms["cbar"][i] - full["cbar"][t]) < 1e-9 * max(1, abs(full["cbar"][t]))
    assert abs(ms["obj"] - full["obj"]) < 1e-9 * max(1, abs(full["obj"]))
    # the master multiplier of stage i is minus the original lam at t_{i+1}
    for i in range(len(bounds) - 2):
        np.testing.assert_allclose(ms["w"][i], -full["lam"][bounds[i + 1]], rtol=1e-8, atol=1e-8)


def test_two_level_tree_equals_original():
    """Reducing the master problem once more (a tree of depth 2) still
    reproduces the original solution at the coarse boundaries."""
    prob = W.g2(3, 2, 24, seed=77)
    full = riccati.solve(prob, want_factors=True)
    b0 = list(range(0, 24, 3)) + [24]                # 8 leaves of length 3
    m1 = reduction.master_problem(prob, b0)          # 7 stages + terminal
    b1 = [0, 3, 6, 7]                                # groups of master stages
    m2 = reduction.master_problem(m1, b1)
    s2 = riccati.solve(m2, want_factors=True)
    for i, s in enumerate(b1[:-1]):
        t = b0[s]
        np.testing.assert_allclose(s2["x"][i], full["x"][t], rtol=1e-8, atol=1e-8)
        np.testing.assert_allclose(s2["P"][i], full["P"][t], rtol=1e-8, atol=1e-8)


def _zero_inputs(prob, t0, t1):
    q = dict(prob)
    q["B"] = np.array(prob["B"], copy=True)
    q["B"][t0:t1] = 0.0
    if q.get("Qxw") is not None:
        q["Qxw"] = np.array(q["Qxw"], copy=True)
        q["Qxw"][t0:t1] = 0.0
    return q


@pytest.mark.parametrize("nx,nu,N,Ns,gap", [(6, 1, 12, 2, None), (8, 2, 17, 3, None), (5, 1, 10, 1, None),
                                            (4, 2, 12, 4, None), (6, 2, 16, 4, (4, 8))])
def test_rank_revealing_master_equals_original(nx, nu, N, Ns, gap):
    """Master problem with the U_1 basis (eqs. Bh_def, Gh_Hh_def): stage i has
    n_uo = rank(S') inputs (min(N_s n_u, n_x) for generic data; 0 for a
    subinterval whose inputs act on nothing), and the master solution still
    gives x_hat_i = x_{t_i}, lam_hat_i = lam_{t_i} and the optimal value of
    P(N), also where the reduced input weight of the plain form is singular."""
    prob = W.with_costs(W.g2(nx, nu, N, seed=N * 3 + nx), seed=4)
    if gap is not None:
        prob = _zero_inputs(prob, *gap)
    full = riccati.solve(prob, want_factors=True)
    bounds = list(range(0, N, Ns)) + [N]
    m = reduction.master_problem_rr(prob, bounds)
    for i, s in enumerate(m["stages"]):
        want = min(Ns * nu, nx)
        if gap is not None and gap[0] <= bounds[i] and bounds[i + 1] <= gap[1]:
            want = 0
        assert s["nuo"] == want
        assert s["B"].shape == (nx, want) and s["Qw"].shape == (want, want)
        if want:
            assert np.linalg.eigvalsh(s["Qw"]).min() > 0
        # the plain form S Qbar^{-1} S' has rank n_uo: singular when n_uo < n_x
        plain = reduction.reduce_closed_form(reduction.sub_problem(prob, bounds[i], bounds[i + 1]))["Qw"]
        ev = np.linalg.eigvalsh(plain)
        assert np.sum(ev > 1e-9 * max(1.0, ev.max())) == want
    ms = reduction.solve_master_dense(m)
    for i, t in enumerate(bounds[:-1]):
        np.testing.assert_allclose(ms["x"][i], full["x"][t], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(ms["lam"][i], full["lam"][t], rtol=1e-8, atol=1e-8)
    assert abs(ms["obj"] - full["obj"]) < 1e-9 * max(1, abs(full["obj"]))


def test_rank_revealing_stage_depends_on_B_Qinv_Bt_only():
    """B_hat Qw_hat^{-1} B_hat' of the U_1 stage equals the plain form's
    S Qbar^{-1} S', and a master whose stages take any other factor of that
    matrix as B with Q_w = I (here one from an eigendecomposition) has the same
    solution: the input parametrisation of a master stage does not matter."""
    nx, nu, N, Ns = 6, 1, 12, 2
    prob = W.with_costs(W.g2(nx, nu, N, seed=41), seed=6)
    full = riccati.solve(prob)
    bounds = list(range(0, N, Ns)) + [N]
    m = reduction.master_problem_rr(prob, bounds)
    for i, s in enumerate(m["stages"]):
        plain = reduction.reduce_closed_form(reduction.sub_problem(prob, bounds[i], bounds[i + 1]))["Qw"]
        M = s["B"] @ np.linalg.solve(s["Qw"], s["B"].T)
        np.testing.assert_allclose(M, plain, rtol=1e-9, atol=1e-11 * np.abs(plain).max())
        ev, U = np.linalg.eigh(plain)
        keep = ev > 1e-9 * ev.max()
        s["B"] = U[:, keep] * np.sqrt(ev[keep])
        s["Qw"] = np.eye(int(keep.sum()))
        s["nuo"] = int(keep.sum())
    ms = reduction.solve_master_dense(m)
    for i, t in enumerate(bounds[:-1]):
        np.testing.assert_allclose(ms["x"][i], full["x"][t], rtol=1e-9, atol=1e-9)
    assert abs(ms["obj"] - full["obj"]) < 1e-9 * max(1, abs(full["obj"]))


@pytest.mark.parametrize("nx,nu,N", [(3, 2, 6), (4, 2, 9), (2, 3, 4)])
def test_linearised_terminal_gives_the_same_solution(nx, nu, N):
    """A subproblem with terminal cost 1/2 x'P_hat x - Psi_hat'x and the one
    whose terminal cost is the linear lam_N'x_N, lam_N = P_hat x_N* - Psi_hat
    taken at its optimum, have the same solution (the KKT conditions coincide
    at that point and both problems are strictly convex in the inputs): the
    down passes solve every leaf and master subproblem below the top this
    way, with the preliminary factorization (P_N = 0) and lam_N from the
    parent."""
    rng = np.random.default_rng(nx * 17 + N)
    prob = W.with_costs(W.g2(nx, nu, N, seed=N + 3), seed=1)
    Ph, Psih, ch = _terminal(rng, nx)
    sub = reduction.sub_problem(prob, 0, N, terminal=(Ph, Psih, ch))
    sub["x0"] = rng.standard_normal(nx)
    full = riccati.solve(sub)
    lamN = Ph @ full["x"][N] - Psih
    lin = dict(sub)
    lin["QxN"], lin["lN"], lin["cN"] = np.zeros((nx, nx)), lamN, 0.0
    sol = riccati.solve(lin)
    for k in ("x", "w", "lam"):
        np.testing.assert_allclose(sol[k], full[k], rtol=1e-9, atol=1e-10)
