"""GPU parity: the HIP parallel Riccati solve (through the C ABI) against the
serial FP64 oracle, element by element on (x, w, lam) and on the optimal value.
Tolerance: relative error <= 1e-10 per block (FP64 path)."""
import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _rs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import rs
    return torch, rs


def _solve_gpu(probs, **opt):
    torch, rs = _rs()
    data = {k: [p[k] for p in probs] for k in probs[0]}
    b = rs.Batch(data, **opt)
    b.solve()
    torch.cuda.synchronize()
    st = b.status()
    out = [b.result(i) for i in range(len(probs))]
    b.close()
    return out, st


def _check(prob, sol, tol=TOL):
    ref = riccati.solve(prob)
    err = kkt.rel_error(sol, ref)
    assert err <= tol, "rel err %.3e" % err
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))
    return err


@pytest.mark.parametrize("Ns", [2, 4, 8, 16, 64])
def test_small_config_g1(Ns):
    """n_x=4, n_u=2, N=64 (G1), every leaf length, several tree depths."""
    prob = W.with_costs(W.g1(4, 2, 64, seed=W.seed_for(0)), seed=1)
    (sol,), st = _solve_gpu([prob], Ns=Ns, branch=2)
    assert st[0, 0] == 0
    _check(prob, sol)


@pytest.mark.parametrize("N,Ns,b", [(1, 4, 2), (5, 4, 2), (37, 4, 3), (100, 8, 2), (33, 2, 4),
                                    (16, 4, 4), (17, 4, 4), (200, 3, 5)])
def test_ragged_and_degenerate_trees(N, Ns, b):
    prob = W.with_costs(W.g2(4, 2, N, seed=N * 3 + Ns), seed=N)
    (sol,), st = _solve_gpu([prob], Ns=Ns, branch=b)
    assert st[0, 0] == 0
    _check(prob, sol)


@pytest.mark.parametrize("nx,nu", [(1, 1), (2, 1), (2, 2), (3, 2), (6, 3), (8, 4), (16, 8), (16, 16), (32, 16), (32, 32)])
def test_shapes(nx, nu):
    prob = W.g2(nx, nu, 96, seed=nx * 10 + nu)
    Ns = max(4, -(-nx // nu))
    (sol,), st = _solve_gpu([prob], Ns=Ns, branch=3)
    assert st[0, 0] == 0
    _check(prob, sol)


@pytest.mark.parametrize("Ns", [4, 8, 16, 32, 64])
def test_config2_full_size(Ns):
    """n_x=20, n_u=10, N=1024, G2 with cross term; leaf length swept 4..64."""
    prob = W.g2(20, 10, 1024, seed=W.seed_for(1))
    (sol,), st = _solve_gpu([prob], Ns=Ns, branch=4)
    assert st[0, 0] == 0
    _check(prob, sol)


def test_headline_shape_full_size():
    """n_x=32, n_u=16, N=1024 (the headline metric's shape)."""
    prob = W.g2(32, 16, 1024, seed=W.seed_for(5))
    (sol,), st = _solve_gpu([prob], Ns=16, branch=4)
    assert st[0, 0] == 0
    _check(prob, sol)


def test_batch_mixed_shapes_and_lengths():
    """A batch mixing shapes and horizons; every instance matches the oracle
    and equals its solve alone (the plan of an instance does not depend on
    the other instances of the batch)."""
    rng = np.random.default_rng(3)
    probs = []
    for i in range(12):
        nx, nu = [(4, 2), (8, 4), (16, 8)][i % 3]
        N = int(rng.integers(1, 300))
        probs.append(W.g2(nx, nu, N, seed=1000 + i))
    sols, st = _solve_gpu(probs, Ns=8, branch=4)
    assert np.all(st[:, 0] == 0)
    for p, s in zip(probs, sols):
        _check(p, s)
    alone, _ = _solve_gpu([probs[5]], Ns=8, branch=4)
    for k in ("x", "w", "lam"):
        np.testing.assert_array_equal(alone[0][k], sols[5][k])


def test_result_invariant_to_tree_shape():
    """The method is exact: leaf length and branch change rounding only."""
    prob = W.g2(8, 4, 300, seed=9)
    ref, _ = _solve_gpu([prob], Ns=4, branch=2)
    for Ns, b in ((8, 3), (16, 4), (300, 2), (2, 8)):
        sol, _ = _solve_gpu([prob], Ns=Ns, branch=b)
        assert kkt.rel_error(sol[0], ref[0]) < 1e-11


def test_time_invariant_stride_zero():
    """Matrices given once with stage stride 0 equal their materialised copy."""
    prob = W.g1(4, 2, 50, seed=2)
    torch, rs = _rs()
    data = {k: [v] for k, v in prob.items()}
    for k in ("A", "B"):
        data[k] = [prob[k][:1]]
    b = rs.Batch(data, Ns=4, branch=2)
    b.solve()
    torch.cuda.synchronize()
    _check(prob, b.result(0))
    b.close()


def test_not_spd_reported_with_stage():
    prob = W.g1(4, 2, 40, seed=4)
    prob["Qw"] = prob["Qw"].copy()
    prob["Qw"][13] = -5.0 * np.eye(2)
    prob["B"] = prob["B"].copy()
    prob["B"][13] = 0.0
    _, st = _solve_gpu([prob], Ns=4, branch=2)
    assert st[0, 0] == 2 and st[0, 1] == 13


def test_repeated_calls_same_workspace():
    """Epoch-tagged tree flags: back-to-back solves on one workspace agree."""
    torch, rs = _rs()
    prob = W.g2(8, 4, 257, seed=12)
    data = {k: [v] for k, v in prob.items()}
    b = rs.Batch(data, Ns=4, branch=2)
    outs = []
    for _ in range(3):
        b.solve()
        torch.cuda.synchronize()
        outs.append(b.result(0))
    b.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o["x"], outs[0]["x"])
    _check(prob, outs[0])


def test_batching_config_uneven_horizons_sampled():
    """4096 instances of n_x=16, n_u=8 with horizons uniform in [32, 2048]
    (G1), one launch per kernel kind; sampled instances (first, last and
    seeded picks, the shortest and the longest) against the oracle."""
    torch, rs = _rs()
    rng = np.random.default_rng(W.seed_for(2))
    Ns_all = rng.integers(32, 2049, size=4096)
    probs = [W.g1_invariant(16, 8, int(n), seed=W.seed_for(2, i)) for i, n in enumerate(Ns_all)]
    data = {k: [p[k] for p in probs] for k in probs[0]}
    b = rs.Batch(data, Ns=16, branch=4)        # A, B, Qxw with stage stride 0
    b.solve()
    torch.cuda.synchronize()
    st = b.status()
    assert np.all(st[:, 0] == 0)
    pick = sorted({0, 4095, int(np.argmin(Ns_all)), int(np.argmax(Ns_all))} |
                  set(int(i) for i in rng.integers(0, 4096, size=60)))
    for i in pick:
        _check(W.materialize(probs[i]), b.result(i))
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_headline_batch_in_the_bench_launch_configuration(precision):
    """The benchmarked workload at full size: 1024 instances of n_x = 32,
    n_u = 16, N = 1024 (G2 drawn on the device, the bench's seed), leaf
    length 512 and branch 8, FP64 and mixed.  Every instance reports success
    (mixed: converged), and sampled instances match the serial oracle at
    1e-10 (the oracle needs about a second per instance, so not all 1024)."""
    torch, rs = _rs()
    data = W.g2_torch(32, 16, 1024, 1024, seed=W.seed_for(5), device="cuda")
    bt = rs.Batch(data, precision=precision, Ns=512, branch=8)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    if precision == 1:
        st = bt.refine_stats()
        assert np.all(st[:, 3] == 1.0) and st[:, 0].max() <= TOL
    rng = np.random.default_rng(11)
    for i in sorted({0, 511, 1023} | set(int(j) for j in rng.integers(0, 1024, size=3))):
        _check(W.instance_to_numpy(data, i), bt.result(i))
    bt.close()
    del data
    torch.cuda.empty_cache()
