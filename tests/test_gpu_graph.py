"""HIP-graph capture of whole calls and per-instance plans.

Each graph is replayed several times with eager work (other solves, torch
kernels, synchronizations) between the replays, and every replay is compared
with the eager result of the same call."""
import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import rs
    return torch, rs


def _data(probs):
    return {k: [p[k] for p in probs] for k in probs[0]}


def _snapshot(bt):
    return [bt.result(i) for i in range(bt.count)], bt.status().copy()


def _same(a, b):
    for ra, rb in zip(a, b):
        for k in ("x", "w", "lam"):
            np.testing.assert_array_equal(ra[k], rb[k])
        assert ra["obj"] == rb["obj"]


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_eager(precision):
    torch, rs = _rs()
    probs = [W.g2(32, 16, n, seed=70 + n) for n in (64, 200, 333)]
    other = [W.g2(16, 16, 90, seed=5)]
    bt = rs.Batch(_data(probs), precision=precision, Ns=8, branch=3)
    ot = rs.Batch(_data(other), precision=precision, Ns=4, branch=2)
    bt.solve()
    torch.cuda.synchronize()
    eager, st = _snapshot(bt)
    assert np.all(st[:, 0] == 0)
    g = bt.capture(0)
    for rep in range(3):
        for t in bt.x + bt.w + bt.lam:
            t.fill_(float("nan"))          # a replay must rewrite everything
        bt.obj.fill_(0.0)
        bt.replay(g)
        torch.cuda.synchronize()
        res, st2 = _snapshot(bt)
        _same(res, eager)
        assert np.array_equal(st2, st)
        ot.solve()                         # eager work between the replays
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
    for p, r in zip(probs, eager):
        assert kkt.rel_error(r, riccati.solve(p)) <= 1e-10
    bt.close()
    ot.close()


def test_factor_and_solve_graphs_with_changing_rhs():
    torch, rs = _rs()
    prob = W.g2(32, 16, 256, seed=31)
    bt = rs.Batch(_data([prob]), Ns=8, branch=4, factored=True)
    gf = bt.capture(1)
    gs = bt.capture(2)
    bt.replay(gf)
    rng = np.random.default_rng(2)
    for r in range(3):
        q = dict(prob)
        for k in ("x0", "a", "lx", "lw", "c", "lN", "cN"):
            q[k] = rng.standard_normal(np.shape(prob[k]))
            bt.update(k, 0, q[k])
        bt.replay(gs)
        torch.cuda.synchronize()
        got = bt.result(0)
        bt.solve_factored()                # eager call, same factors
        torch.cuda.synchronize()
        _same([got], [bt.result(0)])
        assert kkt.rel_error(got, riccati.solve(q)) <= 1e-10
    bt.close()


def test_per_instance_plans_are_batch_independent():
    """Leaf length and branch chosen per instance: every instance equals its
    solve alone bit for bit and matches the oracle."""
    torch, rs = _rs()
    probs = [W.g2(16, 16, 300, seed=1), W.g2(32, 16, 77, seed=2), W.g2(32, 32, 150, seed=3),
             W.g2(16, 16, 41, seed=4)]
    per = [(4, 2), (16, 4), (8, 3), (32, 2)]
    for precision in (0, 1):
        bt = rs.Batch(_data(probs), precision=precision, per_instance=per)
        bt.solve()
        torch.cuda.synchronize()
        assert np.all(bt.status()[:, 0] == 0)
        for i, p in enumerate(probs):
            one = rs.Batch(_data([p]), precision=precision, per_instance=[per[i]])
            one.solve()
            torch.cuda.synchronize()
            _same([bt.result(i)], [one.result(0)])
            one.close()
            assert kkt.rel_error(bt.result(i), riccati.solve(p)) <= 1e-10
        bt.close()
