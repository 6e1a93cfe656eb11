"""RS_PROB_SKIP: an excluded instance is not touched (outputs keep their
contents) while the others are solved exactly as without the exclusion."""
import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,shapes", [(0, [(32, 16), (16, 16), (32, 32)]), (1, [(32, 16), (16, 16)]),
                                              (0, [(4, 2), (8, 4)]), (0, [(16, 8), (32, 4)]), (1, [(16, 8), (32, 8)])])
def test_skipped_instances_untouched(precision, shapes):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import rs
    probs = []
    for i in range(6):
        nx, nu = shapes[i % len(shapes)]
        probs.append(W.g2(nx, nu, 60 + 37 * i, seed=900 + i))
    data = {k: [p[k] for p in probs] for k in probs[0]}
    bt = rs.Batch(data, precision=precision, Ns=8, branch=3)
    full = rs.Batch(data, precision=precision, Ns=8, branch=3)
    full.solve()
    skip = {1, 4}
    for i in skip:
        bt.set_skip(i)
        bt.x[i].fill_(7.0)
        bt.w[i].fill_(7.0)
        bt.lam[i].fill_(7.0)
    bt.solve()
    torch.cuda.synchronize()
    st = bt.status()
    for i, p in enumerate(probs):
        if i in skip:
            r = bt.result(i)
            assert np.all(r["x"] == 7.0) and np.all(r["w"] == 7.0) and np.all(r["lam"] == 7.0)
        else:
            assert st[i, 0] == 0
            for k in ("x", "w", "lam"):
                np.testing.assert_array_equal(bt.result(i)[k], full.result(i)[k])
            assert kkt.rel_error(bt.result(i), riccati.solve(p)) <= 1e-10
    # re-enabled, the skipped instances solve normally on the same plan
    for i in skip:
        bt.set_skip(i, False)
    bt.solve()
    torch.cuda.synchronize()
    for i in skip:
        assert kkt.rel_error(bt.result(i), riccati.solve(probs[i])) <= 1e-10
    bt.close()
    full.close()
