"""GPU parity of the rank-revealing master stages (RS_PLAN_RANK_REVEAL, the
reduction with a basis of range(S') of Sec. 4.2): leaves with
Ns * nu < nx (down to Ns = 1), a stretch of stages whose inputs act on
nothing (a leaf of rank 0), every kernel family (fused matrix-core shapes,
generic small shapes, large-block shapes), FP64 and mixed precision, the
stored factorization with several right-hand sides and a receding-horizon
plan.  Every solution matches the serial FP64 oracle on the full problem
(relative error <= 1e-10 per block); with full-rank leaves the flag changes
nothing beyond rounding."""
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


def _no_inputs(prob, t0, t1):
    q = dict(prob)
    q["B"] = np.array(prob["B"], copy=True)
    q["B"][t0:t1] = 0.0
    q["Qxw"] = np.array(prob["Qxw"], copy=True)
    q["Qxw"][t0:t1] = 0.0
    return q


def _check(prob, sol, tol=TOL):
    ref = riccati.solve(prob)
    err = kkt.rel_error(sol, ref)
    assert err <= tol, "rel err %.3e" % err
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))
    return err


def _run(probs, **opt):
    torch, rs = _rs()
    data = {k: [p[k] for p in probs] for k in probs[0]}
    bt = rs.Batch(data, rank_reveal=True, **opt)
    bt.solve()
    torch.cuda.synchronize()
    return rs, bt


@pytest.mark.parametrize("nx,nu,N,Ns,b", [
    (32, 16, 100, 1, 4),      # fused matrix-core shape, one stage per leaf (rank 16 < 32)
    (16, 16, 90, 1, 3),       # full-rank leaves: the flag only changes the master parametrisation
    (32, 32, 70, 1, 4),
    (20, 10, 64, 1, 4),       # generic shapes
    (4, 2, 50, 1, 2),
    (6, 1, 40, 2, 4),
    (64, 16, 48, 2, 4),       # large-block shapes
    (128, 64, 24, 1, 4),
    (48, 8, 60, 3, 3),
])
def test_rank_revealing_fp64_matches_oracle(nx, nu, N, Ns, b):
    prob = W.with_costs(W.g2(nx, nu, N, seed=nx * 5 + nu + N), seed=Ns)
    rs, bt = _run([prob], Ns=Ns, branch=b)
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    bt.close()


@pytest.mark.parametrize("nx,nu,N,Ns,b,gap", [(32, 16, 200, 8, 4, (16, 40)), (16, 8, 120, 4, 3, (8, 20)),
                                              (20, 10, 80, 4, 2, (4, 12)), (64, 32, 64, 4, 3, (8, 20))])
def test_leaf_without_effective_inputs(nx, nu, N, Ns, b, gap):
    """B_t = 0 (and Q_xw,t = 0) over whole leaves: their reduced input weight
    is zero (rank 0), which the plain form cannot factor; the rank-revealing
    master stage has B = 0, Q_w = I and the solution is still exact."""
    prob = _no_inputs(W.with_costs(W.g2(nx, nu, N, seed=nx + N + 9), seed=2), *gap)
    rs, bt = _run([prob], Ns=Ns, branch=b)
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    bt.close()


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(32, 16, 150, 1, 4), (16, 8, 96, 1, 4), (64, 16, 40, 2, 4),
                                          (20, 10, 60, 1, 3)])
def test_rank_revealing_mixed_matches_oracle_after_refinement(nx, nu, N, Ns, b):
    """FP32 leaves (the rank decision taken on the FP32 reduced weight with
    the FP32 unit roundoff), FP64 master levels and refinement to 1e-10."""
    torch, rs = _rs()
    prob = W.g2(nx, nu, N, seed=3 * N + nx)
    rs, bt = _run([prob], precision=rs.RS_MIXED_FP32, Ns=Ns, branch=b)
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    st = bt.refine_stats()[0]
    assert st[3] == 1.0 and st[0] <= TOL
    bt.close()


def test_rank_revealing_batch_of_mixed_shapes_and_horizons():
    probs = [W.g2(32, 16, n, seed=600 + n) for n in (1, 7, 33, 100)]
    probs += [W.g2(8, 2, 45, seed=650), W.g2(64, 32, 30, seed=651), W.g2(4, 1, 21, seed=652)]
    rs, bt = _run(probs, Ns=2, branch=3)
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        _check(p, bt.result(i))
    bt.close()


def test_rank_revealing_factor_then_several_solves():
    torch, rs = _rs()
    prob = W.g2(32, 16, 120, seed=701)
    data = {k: [prob[k]] for k in prob}
    bt = rs.Batch(data, Ns=1, branch=4, factored=True, rank_reveal=True)
    bt.factor()
    rng = np.random.default_rng(7)
    for r in range(2):
        q = dict(prob)
        for k in RHS_KEYS:
            q[k] = rng.standard_normal(np.shape(prob[k]))
            bt.update(k, 0, q[k])
        bt.solve_factored()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        _check(q, bt.result(0))
    bt.close()


def test_full_rank_leaves_same_solution_with_and_without_flag():
    torch, rs = _rs()
    prob = W.with_costs(W.g2(32, 16, 256, seed=801), seed=8)
    data = {k: [prob[k]] for k in prob}
    sols = []
    for rr in (False, True):
        bt = rs.Batch(data, Ns=8, branch=4, rank_reveal=rr)
        bt.solve()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        sols.append(bt.result(0))
        bt.close()
    assert kkt.rel_error(sols[1], sols[0]) <= 1e-11
