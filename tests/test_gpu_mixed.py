"""GPU parity of the mixed-precision path (FP32 leaf factorization, FP64
master levels, FP64 KKT residual and iterative refinement) against the serial
FP64 oracle: the refined solution must meet the FP64 path's bound, relative
error <= 1e-10, and the refinement statistics must show that it did."""
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
    return torch, rs, rs.Batch(data, precision=rs.RS_MIXED_FP32, **opt)


def _check(prob, sol, tol=TOL):
    ref = riccati.solve(prob)
    err = kkt.rel_error(sol, ref)
    assert err <= tol, "rel err %.3e" % err
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))
    return err


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(32, 16, 300, 8, 4), (16, 16, 97, 4, 3), (32, 32, 64, 4, 2),
                                          (32, 16, 1024, 16, 4), (16, 16, 12, 16, 2)])
def test_mixed_matches_oracle_after_refinement(nx, nu, N, Ns, b):
    prob = W.g2(nx, nu, N, seed=7 * N + nx)
    torch, rs, bt = _batch([prob], Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    st = bt.refine_stats()[0]
    assert st[3] == 1.0                 # converged
    assert st[0] <= TOL                 # relative KKT residual of the result
    assert st[1] <= 0.1 * TOL           # estimated forward error
    assert 1 <= st[2] <= 5              # corrections applied
    bt.close()


def test_refinement_is_needed_and_contracts():
    """The FP32 factorization alone is far from 1e-10 (the first correction is
    large); each correction contracts the error.  A target below what one
    correction reaches, with a single correction allowed, is reported as
    RS_ERR_NOT_CONVERGED; with more corrections the estimate keeps falling."""
    prob = W.g2(32, 16, 256, seed=3)
    ref = riccati.solve(prob)
    torch, rs, bt = _batch([prob], Ns=8, branch=4, max_refine=1, tol=1e-15)
    bt.solve()
    torch.cuda.synchronize()
    st1 = bt.refine_stats()[0]
    assert bt.status()[0, 0] == rs.RS_ERR_NOT_CONVERGED
    assert st1[2] == 1 and st1[4] > 1e-9     # first correction large: FP32 factors
    err1 = kkt.rel_error(bt.result(0), ref)
    assert err1 < 1e-9                       # one correction already contracts it
    bt.close()
    torch, rs, bt = _batch([prob], Ns=8, branch=4, max_refine=3, tol=1e-15)
    bt.solve()
    torch.cuda.synchronize()
    st3 = bt.refine_stats()[0]
    assert st3[2] >= 2 and st3[4] < st1[4] * 1e-3
    assert kkt.rel_error(bt.result(0), ref) <= err1
    bt.close()


def test_mixed_batch_and_alone_identical():
    """Heterogeneous batch: every instance meets the bound, and an instance
    solved alone is bit-identical to the same instance in the batch."""
    rng = np.random.default_rng(11)
    probs = []
    for i in range(9):
        nx, nu = [(16, 16), (32, 16), (32, 32)][i % 3]
        probs.append(W.g2(nx, nu, int(rng.integers(8, 400)), seed=500 + i))
    torch, rs, bt = _batch(probs, Ns=8, branch=3)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        _check(p, bt.result(i))
    mixed_res = bt.result(4)
    bt.close()
    torch, rs, one = _batch([probs[4]], Ns=8, branch=3)
    one.solve()
    torch.cuda.synchronize()
    alone = one.result(0)
    for k in ("x", "w", "lam"):
        np.testing.assert_array_equal(alone[k], mixed_res[k])
    one.close()


def test_mixed_factor_once_solve_many():
    prob = W.g2(32, 16, 200, seed=8)
    torch, rs, bt = _batch([prob], Ns=8, branch=4)
    bt.factor()
    rng = np.random.default_rng(5)
    for r in range(3):
        q = dict(prob)
        for k in RHS_KEYS:
            q[k] = rng.standard_normal(np.shape(prob[k]))
            bt.update(k, 0, q[k])
        bt.solve_factored()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        _check(q, bt.result(0))
    bt.close()


def test_mixed_not_spd_is_reported_not_refined():
    prob = W.g1(16, 16, 40, seed=4)
    prob["Qw"] = prob["Qw"].copy()
    prob["Qw"][21] = -5.0 * np.eye(16)
    prob["B"] = prob["B"].copy()
    prob["B"][21] = 0.0
    torch, rs, bt = _batch([prob], Ns=4, branch=2)
    bt.solve()
    torch.cuda.synchronize()
    st = bt.status()
    assert st[0, 0] == rs.RS_ERR_NOT_SPD and st[0, 1] == 21
    assert bt.refine_stats()[0][2] == 0     # nothing refined
    bt.close()
