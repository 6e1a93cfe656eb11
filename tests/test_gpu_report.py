"""Per-instance report (rs_info, RS_PLAN_REPORT) against the oracle.

The report's quantities are those of the KKT system of P(N) (Sec. 3): the
relative residual of the returned solution, the normwise backward error
||r - K z|| / (||K|| ||z|| + ||r||) in infinity norms, and an estimate of
the relative forward error.  The checks form the same quantities on the
host from the oracle's dense KKT matrix (``kkt.assemble``, small N) and
blockwise residual (``kkt.rel_residual``), and the true forward error from
the serial oracle's solution.  Two FP64 evaluations of a residual of a
direct FP64 solve differ by rounding noise of the size of the residual
itself, so there the bar is a multiple of the unit roundoff u = 2^-53
times the scale (||K|| ||z|| + ||r||) / ||r||; for refined mixed-precision
solutions the residual is far above that noise and the two agree closely."""
import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _rs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import rs
    return torch, rs


def _host_measures(prob, sol):
    """rel_resid, bwd_err, ||K||, ||z||, ||r|| of sol, on the host."""
    K, r = kkt.assemble(prob)
    blocks = kkt.residual_blocks(prob, sol["x"], sol["w"], sol["lam"])
    rho = max(np.abs(b).max() for b in blocks if b.size)
    kn = np.abs(K).sum(axis=1).max()
    zn = max(np.abs(sol[k]).max() for k in ("x", "w", "lam"))
    rn = np.abs(r).max()
    return rho / rn, rho / (kn * zn + rn), kn, zn, rn


def _solve(probs, precision, report=True, factored=False, **opt):
    torch, rs = _rs()
    data = {k: [p[k] for p in probs] for k in probs[0]}
    b = rs.Batch(data, precision=precision, report=report, factored=factored, **opt)
    if factored:
        b.factor()
        b.solve_factored()
    else:
        b.solve()
    torch.cuda.synchronize()
    rep = b.report()
    sols = [b.result(i) for i in range(len(probs))]
    st = b.status()
    b.close()
    return rep, sols, st


@pytest.mark.parametrize("nx,nu,N,Ns,br,factored", [(32, 16, 24, 8, 2, False), (16, 16, 30, 4, 3, False),
                                                    (32, 16, 24, 8, 2, True), (64, 32, 12, 4, 2, False),
                                                    (4, 2, 40, 4, 2, False), (20, 10, 24, 4, 2, False)])
def test_report_fp64_matches_host_measures(nx, nu, N, Ns, br, factored):
    _, rs = _rs()
    probs = [W.with_costs(W.g2(nx, nu, N, seed=700 + i), seed=5 + i) for i in range(2)]
    rep, sols, st = _solve(probs, rs.RS_FP64, factored=factored, Ns=Ns, branch=br)
    for i, (prob, sol, r) in enumerate(zip(probs, sols, rep)):
        assert st[i, 0] == 0 and r["status"] == 0 and r["bad_stage"] == -1 and r["refine_iters"] == 0
        rres, bwd, kn, zn, rn = _host_measures(prob, sol)
        scale = (kn * zn + rn) / rn
        assert abs(r["rel_resid"] - rres) <= 256 * U * scale, (r["rel_resid"], rres)
        assert r["rel_resid"] <= 1e-10
        assert 0.0 <= r["bwd_err"] <= 256 * U and abs(r["bwd_err"] - bwd) <= 256 * U
        # forward error estimate: one correction solve, not applied
        err = kkt.rel_error(sol, riccati.solve(prob))
        assert 0.0 <= r["est_fwd_err"] <= 1e-10
        if err > 1e-14:
            assert err / 100 <= r["est_fwd_err"] <= err * 100, (r["est_fwd_err"], err)


@pytest.mark.parametrize("nx,nu,N,Ns,br", [(32, 16, 24, 8, 2), (16, 16, 30, 4, 3), (64, 32, 12, 4, 2),
                                           (8, 4, 40, 4, 2)])
def test_report_mixed_matches_host_measures(nx, nu, N, Ns, br):
    _, rs = _rs()
    probs = [W.with_costs(W.g2(nx, nu, N, seed=800 + i), seed=9 + i) for i in range(2)]
    rep, sols, st = _solve(probs, rs.RS_MIXED_FP32, Ns=Ns, branch=br)
    for i, (prob, sol, r) in enumerate(zip(probs, sols, rep)):
        assert st[i, 0] == 0 and r["status"] == 0
        assert r["refine_iters"] >= 1
        rres, bwd, kn, zn, rn = _host_measures(prob, sol)
        scale = (kn * zn + rn) / rn
        assert r["rel_resid"] <= 1e-10
        assert abs(r["rel_resid"] - rres) <= max(1e-6 * rres, 256 * U * scale), (r["rel_resid"], rres)
        assert abs(r["bwd_err"] - bwd) <= max(1e-6 * bwd, 256 * U), (r["bwd_err"], bwd)
        err = kkt.rel_error(sol, riccati.solve(prob))
        assert err <= 1e-10 and r["est_fwd_err"] <= 1e-11


def test_report_failure_and_no_flag():
    _, rs = _rs()
    good = W.g2(32, 16, 40, seed=901)
    bad = W.g2(32, 16, 40, seed=902)
    bad["Qw"] = np.array(bad["Qw"])
    bad["Qw"][17] = -1e6 * np.eye(16)          # G at stage 17 cannot be positive definite
    rep, sols, st = _solve([good, bad], rs.RS_FP64, Ns=8, branch=2)
    assert rep[0]["status"] == 0 and rep[0]["bad_stage"] == -1
    assert rep[1]["status"] == rs.RS_ERR_NOT_SPD and rep[1]["bad_stage"] == 17
    assert st[1, 0] == rs.RS_ERR_NOT_SPD and st[1, 1] == 17
    # without RS_PLAN_REPORT: FP64 reports the status only, mixed its refinement
    rep, sols, st = _solve([good], rs.RS_FP64, report=False, Ns=8, branch=2)
    assert rep[0]["status"] == 0 and rep[0]["rel_resid"] == -1.0 and rep[0]["bwd_err"] == -1.0
    rep, sols, st = _solve([good], rs.RS_MIXED_FP32, report=False, Ns=8, branch=2)
    assert rep[0]["status"] == 0 and 0.0 < rep[0]["rel_resid"] <= 1e-10 and rep[0]["bwd_err"] == -1.0
    assert rep[0]["refine_iters"] >= 1
