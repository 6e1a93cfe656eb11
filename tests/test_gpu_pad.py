"""GPU parity of instances whose n_u is below the matrix-core tile at
n_x = 16 or 32 (solved with their inputs padded to 16: zero columns in B and
Q_xw, an identity block in Q_w, zero l_w; the padded inputs come out 0 and
only the caller's n_u inputs are written back).  FP64 and mixed precision,
time-invariant B (stage stride 0), absent Q_xw and l_w, plans with chosen
leaf lengths and rank-revealing master stages, the stored factorization, and
batches that mix padded and unpadded shapes.  Relative error <= 1e-10 per
block against the serial FP64 oracle.  Leaf lengths keep Ns * nu >= 2 nx, as
in the other parity tests (at Ns * nu = nx the reduced input weight of a leaf
is nearly singular and an FP32 leaf reduction can make it indefinite)."""
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


def _check(prob, sol, tol=TOL):
    ref = riccati.solve(prob)
    err = kkt.rel_error(sol, ref)
    assert err <= tol, "rel err %.3e" % err
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))


@pytest.mark.parametrize("nx,nu,N,Ns,b,prec", [
    (16, 8, 200, 8, 4, 0), (16, 8, 200, 8, 4, 1), (32, 8, 150, 8, 3, 0), (32, 8, 150, 8, 3, 1),
    (16, 4, 130, 8, 4, 0), (32, 4, 100, 16, 2, 1), (16, 1, 90, 32, 2, 0), (32, 15, 77, 8, 3, 0),
    (16, 8, 7, 16, 4, 0), (16, 8, 1, 4, 2, 1),
])
def test_padded_inputs_match_oracle(nx, nu, N, Ns, b, prec):
    torch, rs = _rs()
    prob = W.with_costs(W.g2(nx, nu, N, seed=nx * 31 + nu + N), seed=b)
    data = {k: [prob[k]] for k in prob}
    bt = rs.Batch(data, precision=prec, Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    sol = bt.result(0)
    assert sol["w"].shape == (N, nu)
    _check(prob, sol)
    if prec == 1:
        st = bt.refine_stats()[0]
        assert st[3] == 1.0 and st[0] <= TOL
    bt.close()


def test_padded_time_invariant_and_absent_terms():
    """G1 data with A, B given once (stride 0); Q_xw and l_w absent."""
    torch, rs = _rs()
    probs = []
    for i, N in enumerate((64, 300, 33)):
        p = W.g1_invariant(16, 8, N, seed=70 + i)
        probs.append(p)
    data = {k: [p[k] for p in probs] for k in probs[0]}
    for k in ("Qxw", "lw"):
        data.pop(k, None)
    bt = rs.Batch(data, Ns=16, branch=4)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        q = dict(W.materialize(p))
        q.pop("Qxw", None)
        q.pop("lw", None)
        _check(q, bt.result(i))
    bt.close()


def test_padded_mixed_with_unpadded_batch_alone_equals_batch():
    torch, rs = _rs()
    probs = [W.g2(16, 8, 120, seed=1), W.g2(32, 16, 90, seed=2), W.g2(32, 8, 64, seed=3), W.g2(20, 10, 50, seed=4),
             W.g2(16, 8, 17, seed=5)]
    data = {k: [p[k] for p in probs] for k in probs[0]}
    bt = rs.Batch(data, Ns=8, branch=3)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        _check(p, bt.result(i))
        one = rs.Batch({k: [v[i]] for k, v in data.items()}, Ns=8, branch=3)
        one.solve()
        torch.cuda.synchronize()
        for k in ("x", "w", "lam"):
            np.testing.assert_array_equal(one.result(0)[k], bt.result(i)[k])
        one.close()
    bt.close()


def test_padded_split_rank_reveal_and_factored():
    torch, rs = _rs()
    lens = [1, 1, 3, 30, 2, 1, 20, 12]          # rank 8..24 of n_x = 16 with n_u = 8
    N = sum(lens)
    prob = W.g2(16, 8, N, seed=8)
    data = {k: [prob[k]] for k in prob}
    bt = rs.Batch(data, split=([lens], [[3, 2]]), rank_reveal=True)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    bt.close()
    rng = np.random.default_rng(9)
    bt = rs.Batch(data, Ns=4, branch=4, factored=True)
    bt.factor()
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
