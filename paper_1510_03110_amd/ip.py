"""Primal-dual interior-point method for P(N) with input bounds
wlo_t <= w_t <= whi_t: the inequality-constrained MHE problem whose search
directions are Newton steps of the form P(N) (Sec. 3).

Mehrotra predictor-corrector.  Every iteration factors the Newton system once
(rs_factor: the matrices change only through Q_w + Sigma) and solves it twice
(rs_solve: the affine predictor and the centring corrector share the
factorization).  Residuals, Q_w + Sigma, the right-hand sides, step lengths
and the update are HIP kernels of the library (rs_ip_*); the host only
decides the centring parameter, the step lengths and termination from a few
reduced scalars.
"""
import ctypes

import numpy as np

from . import rs


class BoxIP:
    """One problem of P(N) (numpy dict, the workloads' layout) with input
    bounds wlo, whi (arrays (N, nu), +-inf for none), solved on the device."""

    def __init__(self, prob, wlo, whi, precision=rs.RS_FP64, Ns=16, branch=4, device="cuda"):
        import torch
        self.torch = torch
        t = lambda v: torch.as_tensor(np.ascontiguousarray(np.asarray(v, dtype=np.float64))).to(device)
        nx, nu = int(prob["QxN"].shape[0]), int(prob["Qw"].shape[-1])
        N = int(np.shape(prob["lx"])[0])
        self.nx, self.nu, self.N = nx, nu, N
        f64 = dict(dtype=torch.float64, device=device)
        self.d = {k: t(prob[k]) for k in ("Qx", "Qw", "Qxw", "A", "B", "a", "lx", "lw", "c", "QxN", "lN", "x0")}
        self.d["cN"] = t(np.atleast_1d(prob.get("cN", 0.0)))
        big = 1e301
        lo = np.nan_to_num(np.broadcast_to(np.asarray(wlo, dtype=np.float64), (N, nu)), neginf=-big, posinf=big)
        hi = np.nan_to_num(np.broadcast_to(np.asarray(whi, dtype=np.float64), (N, nu)), neginf=-big, posinf=big)
        self.lo_h, self.hi_h = lo, hi
        self.wlo, self.whi = t(lo), t(hi)
        z = lambda *shape: torch.zeros(shape, **f64)
        self.x, self.w, self.lam, self.obj = z(N + 1, nx), z(N, nu), z(N + 1, nx), z(1)
        self.ml, self.mu = z(N, nu), z(N, nu)
        self.nQw, self.na, self.nlx, self.nlw, self.nc = z(N, nu, nu), z(N, nx), z(N, nx), z(N, nu), z(N)
        self.nlN, self.nx0, self.ncN = z(nx), z(nx), z(1)
        self.dx, self.dw, self.dlam, self.dobj = z(N + 1, nx), z(N, nu), z(N + 1, nx), z(1)
        self.dw_aff, self.dml, self.dmu = z(N, nu), z(N, nu), z(N, nu)
        self.part, self.stats = z((N + 1) * 8), z(8)
        self.ip = rs.rs_ip()
        ip = self.ip
        ip.nx, ip.nu, ip.N = nx, nu, N
        self._problem(ip.prob, self.d["Qw"], self.d["a"], self.d["lx"], self.d["lw"], self.d["c"], self.d["lN"],
                      self.d["cN"], self.d["x0"], self.x, self.w, self.lam, self.obj)
        self._problem(ip.newton, self.nQw, self.na, self.nlx, self.nlw, self.nc, self.nlN, self.ncN, self.nx0,
                      self.dx, self.dw, self.dlam, self.dobj)
        ip.wlo, ip.swlo, ip.whi, ip.swhi = self.wlo.data_ptr(), nu, self.whi.data_ptr(), nu
        ip.ml, ip.mu = self.ml.data_ptr(), self.mu.data_ptr()
        ip.dw_aff, ip.dml, ip.dmu = self.dw_aff.data_ptr(), self.dml.data_ptr(), self.dmu.data_ptr()
        ip.part, ip.stats = self.part.data_ptr(), self.stats.data_ptr()
        self.plan = rs.rs_plan_create([(nx, nu, N, Ns, branch)], precision=precision, flags=rs.RS_PLAN_FACTORED)
        self.work_bytes = rs.rs_plan_workspace_size(self.plan)
        self.work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device=device)
        self.work_ptr = (self.work.data_ptr() + 255) // 256 * 256
        self.newton = (rs.rs_problem * 1)()
        ctypes.memmove(ctypes.addressof(self.newton), ctypes.addressof(ip.newton), ctypes.sizeof(rs.rs_problem))
        self.info = torch.zeros(2, dtype=torch.int32, device=device)
        # data scale for the residual test
        self.scale = 1.0 + max(float(np.abs(np.asarray(prob[k])).max()) for k in ("lx", "lw", "a", "x0", "lN"))

    def _problem(self, p, Qw, a, lx, lw, c, lN, cN, x0, x, w, lam, obj):
        nx, nu, N, d = self.nx, self.nu, self.N, self.d
        p.nx, p.nu, p.N = nx, nu, N
        for k, bs, src in (("Qx", nx * nx, d["Qx"]), ("Qw", nu * nu, Qw), ("Qxw", nx * nu, d["Qxw"]),
                           ("A", nx * nx, d["A"]), ("B", nx * nu, d["B"])):
            setattr(p, k, src.data_ptr())
            setattr(p, "s" + k, bs)
        p.QxN = d["QxN"].data_ptr()
        for k, v, bs in (("a", a, nx), ("lx", lx, nx), ("lw", lw, nu), ("c", c, 1)):
            setattr(p, k, v.data_ptr())
            setattr(p, "s" + k, bs)
        p.lN, p.cN, p.x0 = lN.data_ptr(), cN.data_ptr(), x0.data_ptr()
        p.x, p.w, p.lam, p.obj = x.data_ptr(), w.data_ptr(), lam.data_ptr(), obj.data_ptr()

    def _call(self, name, *args):
        st = self.torch.cuda.current_stream().cuda_stream
        rs._check(getattr(rs.library(), name)(ctypes.byref(self.ip), *args, st), name)

    def _stats(self):
        return self.stats.cpu().numpy()

    def _init_point(self):
        lo, hi = self.lo_h, self.hi_h
        flo, fhi = lo > -1e300, hi < 1e300
        w0 = np.where(flo & fhi, 0.5 * (lo + hi), np.where(flo, lo + 1.0, np.where(fhi, hi - 1.0, 0.0)))
        self.w.copy_(self.torch.as_tensor(w0))
        self.x.zero_()
        self.lam.zero_()
        self.ml.copy_(self.torch.as_tensor(flo.astype(np.float64)))
        self.mu.copy_(self.torch.as_tensor(fhi.astype(np.float64)))

    def solve(self, tol=1e-9, max_iter=60):
        """Runs the iteration until max residual <= tol * (1 + |data|) and the
        mean complementarity <= tol; returns a dict with x, w, lam, the bound
        multipliers, the iteration count and the final residuals."""
        torch = self.torch
        self._init_point()
        st = self.torch.cuda.current_stream().cuda_stream
        it, hist = 0, []
        while True:
            self._call("rs_ip_newton", 0, 0.0)
            s = self._stats()
            nb = max(s[4], 1.0)
            mu = s[3] / nb
            res = max(s[0], s[1], s[2])
            hist.append((res, mu))
            if (res <= tol * self.scale and mu <= tol) or it >= max_iter:
                break
            rs.rs_factor(self.plan, self.newton, self.work_ptr, self.work_bytes, st, self.info.data_ptr())
            rs.rs_solve(self.plan, self.newton, self.work_ptr, self.work_bytes, st, self.info.data_ptr())
            self._call("rs_ip_step", 0, 0.0)
            s = self._stats()
            ap, ad = float(s[5]), float(s[6])
            self._call("rs_ip_mu", ap, ad)
            s = self._stats()
            sigma = (max(s[7], 0.0) / max(mu * nb, 1e-300)) ** 3 if s[4] > 0 else 0.0
            sigma = min(sigma, 1.0)
            self._call("rs_ip_newton", 1, sigma * mu)
            rs.rs_solve(self.plan, self.newton, self.work_ptr, self.work_bytes, st, self.info.data_ptr())
            self._call("rs_ip_step", 1, sigma * mu)
            s = self._stats()
            ap, ad = min(1.0, 0.99 * float(s[5])), min(1.0, 0.99 * float(s[6]))
            self._call("rs_ip_update", ap, ad)
            it += 1
        torch.cuda.synchronize()
        return dict(x=self.x.cpu().numpy(), w=self.w.cpu().numpy(), lam=self.lam.cpu().numpy(),
                    ml=self.ml.cpu().numpy(), mu=self.mu.cpu().numpy(), iterations=it, history=hist,
                    status=int(self.info[0]))

    def close(self):
        if self.plan is not None:
            rs.rs_plan_destroy(self.plan)
            self.plan = None
