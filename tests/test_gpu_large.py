"""GPU parity of the large-block kernels (n_x, n_u multiples of 16 up to 128
outside the register/LDS-resident shapes: the n_x = 64 serving shape and the
n_x = 128 large-block configuration) against the serial FP64 oracle.  The FP64
solve of these shapes runs on the stored factorization; mixed precision is the
FP32 factorization with FP64 refinement.  Tolerance: relative error <= 1e-10
per block, as for the other shapes."""
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
    return torch, rs, rs.Batch(data, **opt)


def _check(prob, sol, tol=TOL):
    ref = riccati.solve(prob)
    err = kkt.rel_error(sol, ref)
    assert err <= tol, "rel err %.3e" % err
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))
    return err


# (64, 32, 96, 8, 3) is skipped: a run of an experimental register-blocked
# form of the large-block product (since removed from the code) faulted the
# GPU on this case, and the fault's cause was not found.
_FAULTED = pytest.mark.skip(reason="faulted the GPU under a since-removed product variant; cause not found")


@pytest.mark.parametrize("nx,nu,N,Ns,b", [pytest.param(64, 32, 96, 8, 3, marks=_FAULTED), (48, 16, 80, 8, 4), (64, 16, 64, 8, 2),
                                          (16, 32, 40, 4, 3), (128, 64, 48, 4, 3), (96, 48, 50, 8, 2),
                                          (64, 64, 30, 4, 2), (112, 32, 37, 8, 3)])
def test_large_fp64_matches_oracle(nx, nu, N, Ns, b):
    prob = W.with_costs(W.g2(nx, nu, N, seed=nx * 7 + nu + N), seed=N)
    torch, rs, bt = _batch([prob], Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    bt.close()


@pytest.mark.parametrize("refactor", [False, True])
@pytest.mark.parametrize("nx,nu,N,Ns,b,rr,mixed", [(64, 32, 256, 4, 2, False, False),
                                                   (48, 16, 301, 4, 3, True, False),
                                                   (128, 64, 96, 4, 2, False, False),
                                                   (64, 32, 150, 4, 3, False, True)])
def test_large_master_down_pass_forms(nx, nu, N, Ns, b, rr, mixed, refactor):
    """Down pass of the master levels below the top (Alg. 6, k >= 1): the
    superposition sweep on the records of the up pass (default) and the
    second factorization from the parent's message (RS_PLAN_REFACTOR_DOWN),
    on trees of four to six levels with interior and last items, plain and
    rank-revealing master stages, FP64 and mixed.  Both against the oracle,
    and against each other."""
    prob = W.with_costs(W.g2(nx, nu, N, seed=nx + 13 * N), seed=N + 1)
    torch, rs = _rs()
    sols = []
    for flags in ((rs.RS_PLAN_REFACTOR_DOWN if refactor else 0), rs.RS_PLAN_REFACTOR_DOWN):
        _, _, bt = _batch([prob], Ns=Ns, branch=b, rank_reveal=rr, flags=flags,
                          precision=rs.RS_MIXED_FP32 if mixed else rs.RS_FP64)
        bt.solve()
        torch.cuda.synchronize()
        assert bt.status()[0, 0] == 0
        sols.append(bt.result(0))
        bt.close()
    _check(prob, sols[0])
    if not refactor:
        assert kkt.rel_error(sols[0], sols[1]) <= TOL


@pytest.mark.parametrize("N,Ns", [(8, 16), (16, 16), (1, 4)])
def test_large_whole_problem_leaf(N, Ns):
    """A horizon that fits one leaf: Alg. 1-3 on the leaf with the true
    terminal (no master levels)."""
    prob = W.with_costs(W.g2(64, 32, N, seed=300 + N), seed=N)
    torch, rs, bt = _batch([prob], Ns=Ns, branch=2)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    bt.close()


def test_large_uneven_batch_and_mixed_shapes():
    """Instances of several large shapes and horizons in one call, beside a
    register-resident shape (the plan groups them by shape)."""
    probs = [W.g2(64, 32, n, seed=400 + n) for n in (33, 100, 7)]
    probs += [W.g2(32, 16, 50, seed=450), W.g2(48, 32, 41, seed=451)]
    torch, rs, bt = _batch(probs, Ns=8, branch=3)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        _check(p, bt.result(i))
    bt.close()


def test_large_factor_then_several_solves():
    prob = W.g2(64, 32, 120, seed=501)
    torch, rs, bt = _batch([prob], Ns=8, branch=4, factored=True)
    bt.factor()
    rng = np.random.default_rng(5)
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


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(64, 32, 200, 8, 4), (128, 64, 40, 4, 3), (64, 32, 12, 16, 2)])
def test_large_mixed_matches_oracle_after_refinement(nx, nu, N, Ns, b):
    prob = W.g2(nx, nu, N, seed=11 * N + nx)
    torch, rs, bt = _batch([prob], precision=rs_mixed(), Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    st = bt.refine_stats()[0]
    assert st[3] == 1.0 and st[0] <= TOL and 1 <= st[2] <= 5
    bt.close()


def rs_mixed():
    _, rs = _rs()
    return rs.RS_MIXED_FP32


def test_large_not_spd_stage_reported():
    prob = W.g1(64, 32, 40, seed=4)
    prob["Qw"] = prob["Qw"].copy()
    prob["Qw"][13] = -5.0 * np.eye(32)
    prob["B"] = prob["B"].copy()
    prob["B"][13] = 0.0
    torch, rs, bt = _batch([prob], Ns=4, branch=2)
    bt.solve()
    torch.cuda.synchronize()
    st = bt.status()
    assert st[0, 0] == 2 and st[0, 1] == 13
    bt.close()


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(24, 12, 50, 4, 3), (5, 5, 40, 4, 2), (40, 16, 60, 8, 2),
                                          (100, 60, 30, 4, 2), (7, 3, 33, 4, 4)])
def test_large_ragged_shapes_fp64(nx, nu, N, Ns, b):
    """Dimensions that are not multiples of the 16-wide tiles (edge tiles are
    padded with zeros, the diagonal blocks of the Cholesky with the identity)."""
    prob = W.with_costs(W.g2(nx, nu, N, seed=nx * 13 + nu + N), seed=N)
    torch, rs, bt = _batch([prob], Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    bt.close()


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(16, 8, 300, 16, 4), (8, 4, 200, 8, 3), (20, 10, 256, 8, 4),
                                          (4, 2, 64, 4, 2), (24, 12, 10, 16, 2)])
def test_mixed_precision_small_shapes(nx, nu, N, Ns, b):
    """Mixed precision for the shapes whose fused solve has no matrix-core
    form: FP32 factorization by the large-block kernels, FP64 refinement."""
    prob = W.g2(nx, nu, N, seed=17 * N + nx)
    torch, rs, bt = _batch([prob], precision=rs_mixed(), Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    st = bt.refine_stats()[0]
    assert st[3] == 1.0 and st[0] <= TOL and 1 <= st[2] <= 5
    bt.close()


def test_batching_config_mixed_precision_sampled():
    """4096 instances of n_x=16, n_u=8 with horizons uniform in [32, 2048]
    (G1, time-invariant A and B given once) in mixed precision: FP32
    factorization, FP64 master levels and refinement to 1e-10; every instance
    converges and sampled instances match the oracle."""
    torch, rs = _rs()
    rng = np.random.default_rng(W.seed_for(2))
    Ns_all = rng.integers(32, 2049, size=4096)
    probs = [W.g1_invariant(16, 8, int(n), seed=W.seed_for(2, i)) for i, n in enumerate(Ns_all)]
    data = {k: [p[k] for p in probs] for k in probs[0]}
    b = rs.Batch(data, precision=rs.RS_MIXED_FP32, Ns=16, branch=4)
    b.solve()
    torch.cuda.synchronize()
    assert np.all(b.status()[:, 0] == 0)
    st = b.refine_stats()
    assert np.all(st[:, 3] == 1.0) and st[:, 0].max() <= TOL
    pick = sorted({0, 4095, int(np.argmin(Ns_all)), int(np.argmax(Ns_all))} |
                  set(int(i) for i in rng.integers(0, 4096, size=30)))
    for i in pick:
        _check(W.materialize(probs[i]), b.result(i))
    b.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_large_block_config_full_horizon(prec):
    """The large-block configuration's single instance at full size:
    n_x = 128, n_u = 64, N = 16384 (time-varying G2 data drawn on the device).
    The serial oracle needs minutes here, so the check is the property that
    holds at any size: the relative KKT residual of the returned solution,
    evaluated by the oracle's blockwise residual in FP64, is <= 1e-10 (and
    the mixed-precision solves report convergence; BF16 products need more
    corrections)."""
    torch, rs = _rs()
    data = W.g2_torch(128, 64, 16384, 1, seed=W.seed_for(4), device="cuda")
    bt = rs.Batch(data, precision=prec, Ns=64, branch=8)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    sol = bt.result(0)
    if prec >= 1:
        st = bt.refine_stats()[0]
        assert st[3] == 1.0 and st[0] <= TOL
    bt.close()
    prob = W.instance_to_numpy(data, 0)
    del data
    torch.cuda.empty_cache()
    assert kkt.rel_residual(prob, sol["x"], sol["w"], sol["lam"]) <= TOL


@pytest.fixture(scope="module")
def c5_single():
    """The large-block configuration's single instance (n_x = 128, n_u = 64,
    N = 16384; time-varying A_t, time-invariant B, Q, R given once, drawn on
    the device) and its serial FP64 oracle solution, computed once per
    session (about a minute on one host thread)."""
    torch, rs = _rs()
    data = W.c5_torch(128, 64, 16384, 1, seed=W.seed_for(5), device="cuda")
    prob = W.materialize(W.instance_to_numpy(data, 0))
    ref = riccati.solve(prob)
    return data, prob, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_large_block_config_full_horizon_matches_oracle(c5_single, prec):
    """Full-size large-block configuration against the serial oracle, element
    by element: relative error <= 1e-10 on each of x, w, lam in FP64, in mixed
    precision and with BF16 products (after FP64 refinement)."""
    torch, rs = _rs()
    data, prob, ref = c5_single
    bt = rs.Batch(data, precision=prec, Ns=64, branch=8)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    sol = bt.result(0)
    if prec >= 1:
        st = bt.refine_stats()[0]
        assert st[3] == 1.0 and st[0] <= TOL
    bt.close()
    err = kkt.rel_error(sol, ref)
    print("c5 full horizon, precision %d: rel err vs oracle %.3e" % (prec, err))
    assert err <= TOL
    assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))


def test_large_block_config_batch64_sampled():
    """Batch of 64 instances of n_x = 128, n_u = 64 (the configuration's
    batch; horizon 256 so that the oracle finishes in seconds), mixed
    precision; sampled instances against the oracle."""
    torch, rs = _rs()
    data = W.g2_torch(128, 64, 256, 64, seed=W.seed_for(4, 1), device="cuda")
    bt = rs.Batch(data, precision=rs.RS_MIXED_FP32, Ns=16, branch=4)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    st = bt.refine_stats()
    assert np.all(st[:, 3] == 1.0) and st[:, 0].max() <= TOL
    for i in (0, 17, 63):
        _check(W.instance_to_numpy(data, i), bt.result(i))
    bt.close()


@pytest.mark.timeout(1200)
def test_large_block_config_batch64_full_horizon():
    """The large-block configuration's batch at full size: 64 instances of
    n_x = 128, n_u = 64, N = 16384 (A_t per stage, B, Q, R given once: about
    141 GB of FP64 inputs), FP64, leaf length 64, branch 8, with the leaf
    factorization kept for 1024 leaves at a time (leaf_chunk; the whole one
    would need 790 GB).  Every status must be success and four instances
    (first, last and two inside) must match the serial oracle at 1e-10."""
    torch, rs = _rs()
    from concurrent.futures import ThreadPoolExecutor
    torch.cuda.empty_cache()
    data = W.c5_torch(128, 64, 16384, 64, seed=W.seed_for(5, 64), device="cuda")
    bt = rs.Batch(data, precision=rs.RS_FP64, Ns=64, branch=8, leaf_chunk=1024)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    pick = (0, 21, 42, 63)
    sols = [bt.result(i) for i in pick]
    bt.close()
    probs = [W.materialize(W.instance_to_numpy(data, i)) for i in pick]
    del data
    torch.cuda.empty_cache()
    with ThreadPoolExecutor(max_workers=4) as ex:
        refs = list(ex.map(riccati.solve, probs))
    for i, sol, ref in zip(pick, sols, refs):
        err = kkt.rel_error(sol, ref)
        print("c5 batch-64 instance %d: rel err vs oracle %.3e" % (i, err))
        assert err <= TOL


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(128, 64, 40, 4, 3), (64, 32, 200, 8, 4), (48, 16, 64, 8, 2),
                                          (64, 32, 10, 16, 2)])
def test_bf16_products_match_oracle_after_refinement(nx, nu, N, Ns, b):
    """RS_MIXED_BF16: P [A B], A'PA, A'PB, B'PB of the leaf stages on BF16
    matrix cores with FP32 accumulation; refinement in FP64 reaches the same
    1e-10 bound, with more corrections than the FP32 products need."""
    torch, rs = _rs()
    prob = W.g2(nx, nu, N, seed=23 * N + nx)
    _, _, bt = _batch([prob], precision=rs.RS_MIXED_BF16, Ns=Ns, branch=b)
    bt.solve()
    torch.cuda.synchronize()
    assert bt.status()[0, 0] == 0
    _check(prob, bt.result(0))
    st = bt.refine_stats()[0]
    assert st[3] == 1.0 and st[0] <= TOL and 1 <= st[2] <= 20
    bt.close()
