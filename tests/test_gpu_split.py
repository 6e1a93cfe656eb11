"""GPU parity of plans with chosen subinterval lengths and per-level master
group sizes (rs_plan_create_split; Sec. 4.1 subintervals of different
lengths, Alg. 5 batches of any size): every kernel family, FP64 and mixed
precision, batches of instances with different splits, short leaves with
rank-revealing master stages, and the stored factorization.  Solutions match
the serial FP64 oracle (relative error <= 1e-10 per block); a split with
uniform lengths reproduces the uniform plan bit for bit."""
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


def _lens(rng, N, lo, hi):
    out, t = [], 0
    while t < N:
        v = int(min(rng.integers(lo, hi + 1), N - t))
        out.append(v)
        t += v
    if len(out) > 1 and out[-1] < lo:          # keep every leaf but the last >= lo
        out[-2] += out[-1]
        out.pop()
    return out


@pytest.mark.parametrize("nx,nu,N,lo,hi,brs,prec", [
    (32, 16, 300, 2, 40, [3, 5, 2], 0), (32, 16, 300, 2, 40, [3, 5, 2], 1),
    (16, 16, 200, 1, 25, [2, 7], 0), (32, 32, 150, 1, 30, [4], 1),
    (20, 10, 180, 2, 30, [6, 2], 0), (20, 10, 180, 2, 30, [6, 2], 1),
    (4, 2, 120, 2, 17, [2, 3], 0), (64, 32, 120, 2, 20, [3, 4], 0), (64, 32, 120, 2, 20, [3, 4], 1),
    (128, 64, 40, 2, 9, [2, 5], 0),
])
def test_split_plan_matches_oracle(nx, nu, N, lo, hi, brs, prec):
    torch, rs = _rs()
    rng = np.random.default_rng(nx * 1000 + N + prec)
    lens = _lens(rng, N, lo, hi)
    prob = W.with_costs(W.g2(nx, nu, N, seed=nx + N + 3), seed=lo)
    data = {k: [prob[k]] for k in prob}
    bt = rs.Batch(data, precision=prec, split=([lens], [brs]))
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    if prec == 1:
        st = bt.refine_stats()[0]
        assert st[3] == 1.0 and st[0] <= TOL
    bt.close()


def test_split_batch_of_instances_with_different_splits():
    torch, rs = _rs()
    rng = np.random.default_rng(11)
    probs, lens, brs = [], [], []
    for i, (nx, nu, N) in enumerate([(32, 16, 97), (32, 16, 256), (20, 10, 64), (32, 16, 5), (20, 10, 150)]):
        probs.append(W.g2(nx, nu, N, seed=900 + i))
        lens.append(_lens(rng, N, 2, 33))
        brs.append([int(rng.integers(2, 6)) for _ in range(int(rng.integers(1, 4)))])
    data = {k: [p[k] for p in probs] for k in probs[0]}
    bt = rs.Batch(data, split=(lens, brs))
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        _check(p, bt.result(i))
    bt.close()


def test_split_with_uniform_lengths_is_bit_identical_to_uniform_plan():
    torch, rs = _rs()
    N, Ns, b = 300, 16, 4
    prob = W.g2(32, 16, N, seed=77)
    data = {k: [prob[k]] for k in prob}
    lens = [Ns] * (N // Ns) + [N % Ns]
    a = rs.Batch(data, Ns=Ns, branch=b)
    c = rs.Batch(data, split=([lens], [[b]]))
    for bt in (a, c):
        bt.solve()
    torch.cuda.synchronize()
    ra, rc = a.result(0), c.result(0)
    for k in ("x", "w", "lam"):
        np.testing.assert_array_equal(ra[k], rc[k])
    a.close()
    c.close()


def test_split_short_leaves_with_rank_revealing_masters():
    """Leaves of 1..3 stages (rank 16..48 of n_x = 32 with n_u = 16) next to
    long ones."""
    torch, rs = _rs()
    lens = [1, 1, 2, 40, 1, 3, 25, 1, 1, 30, 2, 13]
    N = sum(lens)
    prob = W.g2(32, 16, N, seed=333)
    data = {k: [prob[k]] for k in prob}
    for prec in (0, 1):
        bt = rs.Batch(data, precision=prec, split=([lens], [[3, 2]]), rank_reveal=True)
        bt.solve()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        _check(prob, bt.result(0))
        bt.close()


def test_split_factor_then_several_solves():
    torch, rs = _rs()
    rng = np.random.default_rng(5)
    prob = W.g2(32, 16, 160, seed=444)
    lens = _lens(rng, 160, 2, 30)
    data = {k: [prob[k]] for k in prob}
    bt = rs.Batch(data, factored=True, split=([lens], [[4, 2]]))
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
