"""Interior-point method for P(N) with input bounds on the GPU (one
factorization and two solves of the Newton system per iteration): the result
matches the bound-constrained minimiser of the oracle (condensing +
bounded-variable least squares), stays within the bounds, and without active
bounds reduces to the unconstrained Newton step."""
import numpy as np
import pytest

from oracle import boxqp, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import ip, rs
    return torch, ip, rs


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(1.0, np.abs(np.asarray(b)).max()))


@pytest.mark.parametrize("nx,nu,N,prec", [(6, 3, 40, 0), (6, 3, 40, 1), (16, 8, 60, 0), (4, 2, 64, 1),
                                          (32, 16, 24, 0)])
def test_box_ip_matches_reference(nx, nu, N, prec):
    torch, ip, rs = _ip()
    prob = W.g2(nx, nu, N, seed=900 + nx + N)
    s = np.abs(riccati.solve(prob)["w"]).max()
    lo, hi = np.full((N, nu), -0.5 * s), np.full((N, nu), 0.4 * s)
    ref = boxqp.solve(prob, lo, hi)
    assert np.isclose(ref["w"], lo).any() and np.isclose(ref["w"], hi).any()     # bounds are active
    solver = ip.BoxIP(prob, lo, hi, precision=prec, Ns=8, branch=4)
    r = solver.solve(tol=1e-10)
    solver.close()
    assert r["status"] == 0 and r["iterations"] < 50
    assert np.all(r["w"] >= lo - 1e-12) and np.all(r["w"] <= hi + 1e-12)
    assert _rel(r["w"], ref["w"]) <= 1e-7, _rel(r["w"], ref["w"])
    assert _rel(r["x"], ref["x"]) <= 1e-7
    assert np.all(r["ml"] >= 0) and np.all(r["mu"] >= 0)


def test_box_ip_inactive_bounds_give_the_newton_step():
    torch, ip, rs = _ip()
    prob = W.g2(8, 4, 50, seed=31)
    ref = riccati.solve(prob)
    s = np.abs(ref["w"]).max()
    solver = ip.BoxIP(prob, np.full((50, 4), -10 * s), np.full((50, 4), 10 * s), Ns=8, branch=3)
    r = solver.solve(tol=1e-11)
    solver.close()
    assert _rel(r["w"], ref["w"]) <= 1e-8 and _rel(r["x"], ref["x"]) <= 1e-8


def test_box_ip_one_sided_and_missing_bounds():
    torch, ip, rs = _ip()
    prob = W.g2(6, 3, 30, seed=47)
    s = np.abs(riccati.solve(prob)["w"]).max()
    lo = np.full((30, 3), -np.inf)
    hi = np.full((30, 3), np.inf)
    lo[:, 0] = -0.3 * s                     # lower bound only on input 0
    hi[:, 1] = 0.3 * s                      # upper bound only on input 1; input 2 free
    ref = boxqp.solve(prob, lo, hi)
    solver = ip.BoxIP(prob, lo, hi, Ns=4, branch=4)
    r = solver.solve(tol=1e-10)
    solver.close()
    assert _rel(r["w"], ref["w"]) <= 1e-7 and _rel(r["x"], ref["x"]) <= 1e-7
