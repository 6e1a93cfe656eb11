"""rs_batch_solve_noalloc: the solve on the library's static device scratch
(no workspace argument, no allocation) gives the same results, bit for bit,
as rs_batch_solve with a caller workspace, call after call on one GPU with
different plans sharing the scratch (the second call smaller than the
first); plans too large for the scratch are refused with RS_ERR_NOMEM."""
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


def _both(probs, **opt):
    """Results of rs_batch_solve (caller workspace) and of
    rs_batch_solve_noalloc on the same Batch (same outputs, overwritten)."""
    torch, rs = _rs()
    data = {k: [p[k] for p in probs] for k in probs[0]}
    b = rs.Batch(data, **opt)
    b.solve()
    torch.cuda.synchronize()
    ref = [b.result(i) for i in range(len(probs))]
    st_ref = b.status().copy()
    for t in b.x + b.w + b.lam:
        t.fill_(float("nan"))
    b.obj.fill_(float("nan"))
    b.info.fill_(-7)
    rs.rs_batch_solve_noalloc(b.plan, b.probs, b.stream_ptr(), b.info.data_ptr())
    torch.cuda.synchronize()
    got = [b.result(i) for i in range(len(probs))]
    st = b.status().copy()
    b.close()
    return ref, got, st_ref, st


def _same(ref, got):
    for a, b in zip(ref, got):
        for k in ("x", "w", "lam"):
            np.testing.assert_array_equal(a[k], b[k])
        assert a["obj"] == b["obj"]


def test_noalloc_equals_workspace_call_twice_smaller():
    _, rs = _rs()
    big = [W.g2(32, 16, 300, seed=2000 + i) for i in range(3)]
    ref, got, st0, st1 = _both(big, precision=rs.RS_FP64, Ns=16, branch=4)
    assert np.all(st0[:, 0] == 0)
    np.testing.assert_array_equal(st0, st1)
    _same(ref, got)
    assert kkt.rel_error(got[1], riccati.solve(big[1])) <= 1e-10
    small = [W.g2(16, 16, 50, seed=2100)]
    ref, got, st0, st1 = _both(small, precision=rs.RS_FP64, Ns=8, branch=2)
    np.testing.assert_array_equal(st0, st1)
    _same(ref, got)
    assert kkt.rel_error(got[0], riccati.solve(small[0])) <= 1e-10


@pytest.mark.parametrize("nx,nu,N,prec", [(32, 16, 200, 1), (64, 32, 60, 0), (8, 4, 120, 1), (4, 2, 64, 0)])
def test_noalloc_other_paths(nx, nu, N, prec):
    _, rs = _rs()
    probs = [W.g2(nx, nu, N, seed=2200 + i) for i in range(2)]
    ref, got, st0, st1 = _both(probs, precision=prec, Ns=8, branch=4)
    assert np.all(st0[:, 0] == 0)
    np.testing.assert_array_equal(st0, st1)
    _same(ref, got)


def test_noalloc_plans_alternate_on_shared_scratch():
    torch, rs = _rs()
    pa = [W.g2(32, 16, 100, seed=2300)]
    pb = [W.g2(16, 16, 40, seed=2301)]
    ba = rs.Batch({k: [p[k] for p in pa] for k in pa[0]}, precision=rs.RS_FP64, Ns=8, branch=2)
    bb = rs.Batch({k: [p[k] for p in pb] for k in pb[0]}, precision=rs.RS_FP64, Ns=8, branch=2)
    outs = []
    for b in (ba, bb, ba, bb):
        rs.rs_batch_solve_noalloc(b.plan, b.probs, b.stream_ptr(), b.info.data_ptr())
        torch.cuda.synchronize()
        assert b.status()[0, 0] == 0
        outs.append(b.result(0))
    _same([outs[0]], [outs[2]])
    _same([outs[1]], [outs[3]])
    assert kkt.rel_error(outs[2], riccati.solve(pa[0])) <= 1e-10
    ba.close()
    bb.close()


def test_noalloc_refuses_plans_beyond_the_scratch():
    torch, rs = _rs()
    plan = rs.rs_plan_create([(32, 16, 1024)] * 64, rs.RS_FP64, 16, 4)
    assert rs.rs_plan_workspace_size(plan) > rs.RS_NOALLOC_SCRATCH_BYTES
    probs = (rs.rs_problem * 64)()
    with pytest.raises(rs.RsError) as e:
        rs.rs_batch_solve_noalloc(plan, probs, None, None)
    assert e.value.status == rs.RS_ERR_NOMEM
    rs.rs_plan_destroy(plan)
