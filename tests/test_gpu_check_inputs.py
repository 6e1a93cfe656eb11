"""RS_PLAN_CHECK_INPUTS: non-finite inputs, planted on the host in otherwise
valid problems, give RS_ERR_ARG with the first offending place (-1 for x0,
the stage, N for the terminal data) on the device; clean instances of the
same batch are unaffected and match the oracle, in FP64 (register-resident
and large-block shapes, padded inputs) and mixed precision."""
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


def _planted(nx, nu, N, seed):
    base = [W.g2(nx, nu, N, seed=seed + i) for i in range(6)]
    for p in base:
        for k in list(p):
            p[k] = np.array(p[k], dtype=np.float64)
    base[1]["A"][37 % N, 2, 1] = np.nan            # stage 37
    base[2]["lx"][5, 0] = np.inf                   # stage 5
    base[3]["x0"][1] = np.nan                      # x0: -1
    base[4]["QxN"][0, 0] = -np.inf                 # terminal: N
    base[5]["Qw"][11, 0, 0] = np.nan               # stage 11 (and stage 40 below)
    base[5]["B"][40, 1, 0] = np.nan
    want = [(0, None), (1, 37 % N), (1, 5), (1, -1), (1, N), (1, 11)]
    return base, want


@pytest.mark.parametrize("nx,nu,N,prec", [(32, 16, 64, 0), (32, 16, 64, 1), (64, 32, 48, 0), (32, 8, 64, 0),
                                          (4, 2, 50, 0)])
def test_nonfinite_inputs_reported(nx, nu, N, prec):
    torch, rs = _rs()
    probs, want = _planted(nx, nu, N, seed=3000)
    data = {k: [p[k] for p in probs] for k in probs[0]}
    b = rs.Batch(data, precision=prec, Ns=8, branch=4, check_inputs=True)
    b.solve()
    torch.cuda.synchronize()
    st = b.status()
    for i, (code, stage) in enumerate(want):
        if code == 0:
            assert st[i, 0] == 0
            assert kkt.rel_error(b.result(i), riccati.solve(probs[i])) <= 1e-10
        else:
            assert st[i, 0] == rs.RS_ERR_ARG and st[i, 1] == stage, (i, st[i], stage)
    b.close()
