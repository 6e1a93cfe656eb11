"""GPU parity of the factor / solve split (rs_factor once, rs_solve for one
or several right-hand sides) against the serial FP64 oracle and against the
fused solve.  Tolerance as for the fused path: relative error <= 1e-10."""
import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10
RHS_KEYS = ("x0", "a", "lx", "lw", "c", "lN", "cN")


def _rs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import rs
    return torch, rs


def _batch(probs, **opt):
    torch, rs = _rs()
    data = {k: [p[k] for p in probs] for k in probs[0]}
    return torch, rs.Batch(data, factored=True, **opt)


def _check(prob, sol, tol=TOL):
    ref = riccati.solve(prob)
    err = kkt.rel_error(sol, ref)
    assert err <= tol, "rel err %.3e" % err
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))
    return err


def _new_rhs(prob, seed):
    """Same matrices, fresh right-hand side (a, lx, lw, c, lN, cN, x0)."""
    rng = np.random.default_rng(seed)
    q = dict(prob)
    for k in RHS_KEYS:
        q[k] = rng.standard_normal(np.shape(prob[k]))
    return q


@pytest.mark.parametrize("refactor", [False, True])
@pytest.mark.parametrize("nx,nu,N,Ns,b,rr,mixed", [(32, 16, 512, 4, 2, False, False),
                                                   (16, 16, 301, 4, 3, True, False),
                                                   (32, 32, 257, 4, 2, False, True),
                                                   (32, 16, 600, 8, 3, False, True)])
def test_master_down_pass_forms(nx, nu, N, Ns, b, rr, mixed, refactor):
    """Down pass of the master levels below the top on the matrix-core
    stored factorization: the superposition sweep on the records of the up
    pass (default) and the second factorization from the parent's message
    (RS_PLAN_REFACTOR_DOWN), on trees of four to seven levels with interior
    and last items, plain and rank-revealing master stages, FP64 (factor,
    then solve) and mixed.  Both against the oracle, and against each other."""
    prob = W.with_costs(W.g2(nx, nu, N, seed=3 * N + nx), seed=N + 2)
    torch, rs = _rs()
    sols = []
    for flags in ((rs.RS_PLAN_REFACTOR_DOWN if refactor else 0), rs.RS_PLAN_REFACTOR_DOWN):
        _, bt = _batch([prob], Ns=Ns, branch=b, rank_reveal=rr, flags=flags,
                       precision=rs.RS_MIXED_FP32 if mixed else rs.RS_FP64)
        if mixed:
            bt.solve()
        else:
            bt.factor()
            bt.solve_factored()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        sols.append(bt.result(0))
        bt.close()
    _check(prob, sols[0])
    if not refactor:
        assert kkt.rel_error(sols[0], sols[1]) <= TOL


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(16, 16, 96, 4, 3), (32, 16, 200, 8, 2), (32, 32, 77, 4, 4),
                                          (32, 16, 1024, 16, 4), (16, 16, 13, 16, 2), (16, 16, 17, 4, 2)])
def test_factor_then_solve_matches_oracle(nx, nu, N, Ns, b):
    prob = W.g2(nx, nu, N, seed=N + nx)
    torch, bt = _batch([prob], Ns=Ns, branch=b)
    bt.factor()
    bt.solve_factored()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    sol = bt.result(0)
    _check(prob, sol)
    # the fused solve on the same workspace agrees to rounding: both are within
    # the oracle bound, and their difference is the sum of two FP64 rounding
    # errors taken in different summation orders (~1e-12 over a few hundred
    # stages)
    bt.solve()
    torch.cuda.synchronize()
    fused = bt.result(0)
    assert kkt.rel_error(sol, fused) < 1e-11
    bt.close()


def test_several_right_hand_sides_per_factorization():
    """One rs_factor, then three rs_solve calls with new a, lx, lw, c, lN, cN, x0."""
    prob = W.g2(32, 16, 300, seed=21)
    torch, bt = _batch([prob], Ns=8, branch=4)
    bt.factor()
    for r in range(3):
        q = _new_rhs(prob, 100 + r)
        for k in RHS_KEYS:
            bt.update(k, 0, q[k])
        bt.solve_factored()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        _check(q, bt.result(0))
    bt.close()


def test_batch_of_factored_instances():
    probs = [W.g2(16, 16, n, seed=40 + n) for n in (1, 5, 64, 150, 333)]
    probs += [W.g2(32, 16, n, seed=50 + n) for n in (16, 129)]
    torch, bt = _batch(probs, Ns=8, branch=3)
    bt.factor()
    bt.solve_factored()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        _check(p, bt.result(i))
    bt.close()


def test_factor_reports_not_spd_stage():
    prob = W.g1(16, 16, 40, seed=4)
    prob["Qw"] = prob["Qw"].copy()
    prob["Qw"][13] = -5.0 * np.eye(16)
    prob["B"] = prob["B"].copy()
    prob["B"][13] = 0.0
    torch, bt = _batch([prob], Ns=4, branch=2)
    bt.factor()
    bt.solve_factored()
    torch.cuda.synchronize()
    st = bt.status()
    assert st[0, 0] == 2 and st[0, 1] == 13     # kept by rs_solve
    bt.close()


def test_time_invariant_stride_zero_factored():
    prob = W.g1(16, 16, 50, seed=2)
    torch, rs = _rs()
    data = {k: [v] for k, v in prob.items()}
    for k in ("A", "B"):
        data[k] = [prob[k][:1]]
    bt = rs.Batch(data, Ns=4, branch=2, factored=True)
    bt.factor()
    bt.solve_factored()
    torch.cuda.synchronize()
    _check(prob, bt.result(0))
    bt.close()
