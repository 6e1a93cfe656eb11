"""Receding-horizon plans on the GPU: windows [s, s+N) of one long stage
sequence, shifted by one stage per call on one workspace, so that interior
leaves reuse the factorization an earlier call stored.  Every window's
solution matches the oracle (relative error <= 1e-10) and is bit-identical to
a call that factors everything on a fresh workspace."""
import ctypes

import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10
STAGE_KEYS = ("Qx", "Qw", "Qxw", "A", "B", "a", "lx", "lw", "c")


def _rs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import rs
    return torch, rs


class _Seq:
    """A stage sequence in device memory and the windows over it."""

    def __init__(self, torch, rs, prob, N):
        self.torch, self.rs, self.prob, self.N = torch, rs, prob, N
        self.nx, self.nu = int(prob["QxN"].shape[0]), int(prob["Qw"].shape[-1])
        f64 = dict(device="cuda", dtype=torch.float64)
        self.d = {k: torch.as_tensor(np.asarray(v, dtype=np.float64)).to(**f64).contiguous() for k, v in prob.items()}

    def outputs(self):
        t, f64 = self.torch, dict(device="cuda", dtype=self.torch.float64)
        return dict(x=t.zeros((self.N + 1, self.nx), **f64), w=t.zeros((self.N, self.nu), **f64),
                    lam=t.zeros((self.N + 1, self.nx), **f64), obj=t.zeros(1, **f64))

    def descriptor(self, s, out):
        nx, nu, N, d = self.nx, self.nu, self.N, self.d
        p = (self.rs.rs_problem * 1)()
        q = p[0]
        q.nx, q.nu, q.N = nx, nu, N
        for k, bs in (("Qx", nx * nx), ("Qw", nu * nu), ("Qxw", nx * nu), ("A", nx * nx), ("B", nx * nu)):
            setattr(q, k, d[k].data_ptr() + 8 * s * bs)
            setattr(q, "s" + k, bs)
        for k, bs in (("a", nx), ("lx", nx), ("lw", nu), ("c", 1)):
            setattr(q, k, d[k].data_ptr() + 8 * s * bs)
            setattr(q, "s" + k, bs)
        for k in ("QxN", "lN", "cN", "x0"):
            setattr(q, k, d[k].data_ptr())
        for k in ("x", "w", "lam", "obj"):
            setattr(q, k, out[k].data_ptr())
        return p

    def window(self, s):
        w = {k: np.asarray(self.prob[k])[s:s + self.N] for k in STAGE_KEYS}
        for k in ("QxN", "lN", "cN", "x0"):
            w[k] = self.prob[k]
        return w


def _solve(rs, torch, seq, plan, work, s, out):
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    ptr = (work.data_ptr() + 255) // 256 * 256
    rs.rs_batch_solve(plan, seq.descriptor(s, out), ptr, work.numel() - 256,
                      torch.cuda.current_stream().cuda_stream, info.data_ptr())
    torch.cuda.synchronize()
    return int(info[0])


@pytest.mark.parametrize("prec,nx,nu,N,Ns,rr", [(0, 32, 16, 150, 16, 0), (1, 32, 16, 150, 16, 0), (0, 64, 32, 70, 8, 0),
                                                (1, 16, 8, 90, 8, 0), (0, 16, 16, 40, 16, 0), (1, 64, 32, 50, 8, 0),
                                                (0, 32, 16, 60, 1, 1), (1, 16, 8, 40, 1, 1), (0, 64, 16, 40, 2, 1)])
def test_receding_horizon_reuse(prec, nx, nu, N, Ns, rr):
    """rr: rank-revealing master stages (leaves with Ns * nu < nx); the
    stored M1 messages then hold the rank-revealing factor."""
    torch, rs = _rs()
    flags = rs.RS_PLAN_RANK_REVEAL if rr else 0
    K = 2 * Ns + 3
    seq = _Seq(torch, rs, W.with_costs(W.g2(nx, nu, N + K, seed=nx + N + prec), seed=3), N)
    lo, hi = 0, 0
    # one plan moved along the sequence (odd instantiations: a new plan per
    # window on the same workspace); both keep the stored factorization
    keep = rs.rs_plan_create_ring([(nx, nu, N, Ns, 4, 0, 0, 0)], precision=prec, flags=flags)
    size = rs.rs_plan_workspace_size(keep)
    work = torch.empty(size + 256, dtype=torch.uint8, device="cuda")
    fresh = torch.empty(size + 256, dtype=torch.uint8, device="cuda")
    for s in range(K):
        if s % 2 == 0:
            rs.rs_plan_ring_update(keep, [(nx, nu, N, Ns, 4, s, lo, hi)])
            plan = keep
        else:
            plan = rs.rs_plan_create_ring([(nx, nu, N, Ns, 4, s, lo, hi)], precision=prec, flags=flags)
        try:
            assert rs.rs_plan_workspace_size(plan) == size
            out = seq.outputs()
            assert _solve(rs, torch, seq, plan, work, s, out) == 0
            win = seq.window(s)
            sol = {k: v.cpu().numpy() for k, v in out.items()}
            sol["obj"] = float(sol["obj"][0])
            ref = riccati.solve(win)
            assert kkt.rel_error(sol, ref) <= TOL
            assert abs(sol["obj"] - ref["obj"]) <= 1e-9 * max(1.0, abs(ref["obj"]))
        finally:
            if plan is not keep:
                rs.rs_plan_destroy(plan)
        if s % 4 == 3 or s == K - 1:
            # the same window factored from scratch on a fresh workspace
            plan = rs.rs_plan_create_ring([(nx, nu, N, Ns, 4, s, 0, 0)], precision=prec, flags=flags)
            try:
                out2 = seq.outputs()
                fresh.zero_()
                assert _solve(rs, torch, seq, plan, fresh, s, out2) == 0
                for k in ("x", "w", "lam"):
                    np.testing.assert_array_equal(out[k].cpu().numpy(), out2[k].cpu().numpy())
            finally:
                rs.rs_plan_destroy(plan)
        lo, hi = rs.ring_current_leaves(s, N, Ns, rank_reveal=rr)
    rs.rs_plan_destroy(keep)
