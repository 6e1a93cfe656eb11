"""Serving loop for receding-horizon (MHE) Newton steps on one GPU.

Every session is a UFTOC window of N stages (an MHE problem over the last N
measurements) kept resident in HBM.  A request appends one new stage to its
session and drops the oldest (a receding-horizon shift); the new initial
state is the previous solution's x_1, and the shifted window is solved.

Device layout.  A session stores its stages as records of
E = 2 nx^2 + nu^2 + 2 nx nu + 2 nx + nu + 1 doubles, padded to 64 bytes
(Qx | Qw | Qxw | A | B | a | lx | lw | c) in a buffer of 2N records; the
window is records [start, start + N), described to the solver with the
record length as the stage stride of every field.  A shift writes one record
(a single host-to-device copy from the session's pinned staging buffer) and
advances start; when the window reaches the end of the buffer, its N - 1
surviving records are moved to the front with one device copy, so the cost
per request stays one record on average.

Continuous batching.  The engine keeps a small number of lanes (a stream, a
workspace and a status array each); every session belongs to one lane.  A
launch on a lane solves the lane's sessions whose request is ready; every
other session of the lane carries RS_PROB_SKIP for that call, and each
instance's tree depends only on itself (results are the same alone and in
any mix).  While one lane's launch runs, newly ready sessions of the other
lanes start on their streams, so their work overlaps on the device.  A
session has at most one request in flight (its next window needs this
solution's x_1); later requests for it wait in its queue.

Factorizations across shifts.  Each launch uses a receding-horizon plan
(rs_plan_create_ring): leaf boundaries sit on absolute stage indices, so a
one-stage shift changes only the window's first and last leaves.  The
interior leaves keep their stored factorization (Alg. 4 records and reduced
form) in the lane's workspace from the session's previous request and are
not factored again; the master levels, the vector passes and the leaf
solves run in full.

Admission.  A session is admitted only while the projected HBM footprint of
all admitted sessions (window buffers, solution arrays and their share of
their lane's workspace) stays within a fraction (0.9) of the device memory
that is not already in use when the engine starts.

Latency is measured from a request's arrival (its scheduled time in the
arrival process) to the host's observation of its launch's completion event.
"""
import time
from collections import deque

import sys

import numpy as np

from . import rs
from .autotune import Tuner


def record_len(nx, nu):
    """Doubles per stage record, padded to 64 bytes so records start on a
    64-byte boundary."""
    e = 2 * nx * nx + nu * nu + 2 * nx * nu + 2 * nx + nu + 1
    return (e + 7) // 8 * 8


def record_offsets(nx, nu):
    o, offs = 0, {}
    for k, n in (("Qx", nx * nx), ("Qw", nu * nu), ("Qxw", nx * nu), ("A", nx * nx), ("B", nx * nu),
                 ("a", nx), ("lx", nx), ("lw", nu), ("c", 1)):
        offs[k] = o
        o += n
    return offs


def pack_stage(stage, nx, nu):
    """One stage (dict of Qx, Qw, Qxw, A, B, a, lx, lw, c) as a record."""
    offs = record_offsets(nx, nu)
    r = np.zeros(record_len(nx, nu), dtype=np.float64)
    for k, o in offs.items():
        v = np.asarray(stage.get(k, 0.0), dtype=np.float64).ravel()
        n = {"Qx": nx * nx, "Qw": nu * nu, "Qxw": nx * nu, "A": nx * nx, "B": nx * nu, "a": nx, "lx": nx,
             "lw": nu, "c": 1}[k]
        r[o:o + n] = v if v.size == n else 0.0
    return r


def unpack_window(records, nx, nu, N):
    """Stage arrays of a window from its (N, E) records (host, for checks)."""
    offs = record_offsets(nx, nu)
    shp = {"Qx": (nx, nx), "Qw": (nu, nu), "Qxw": (nx, nu), "A": (nx, nx), "B": (nx, nu), "a": (nx,),
           "lx": (nx,), "lw": (nu,), "c": ()}
    out = {}
    for k, o in offs.items():
        n = int(np.prod(shp[k])) if shp[k] else 1
        out[k] = records[:, o:o + n].reshape((N,) + shp[k])
    return out


class Session:
    """Device-resident window of one receding-horizon problem."""

    def __init__(self, sid, prob, device):
        import torch
        self.sid = sid
        self.nx = int(prob["QxN"].shape[-1])
        self.nu = int(prob["Qw"].shape[-1])
        self.N = int(np.shape(prob["lx"])[0])
        nx, nu, N = self.nx, self.nu, self.N
        self.E = record_len(nx, nu)
        self.cap = 2 * N
        f64 = dict(dtype=torch.float64, device=device)
        host = np.stack([pack_stage({k: prob[k][t] if np.ndim(prob[k]) > 0 else 0.0 for k in
                                     ("Qx", "Qw", "Qxw", "A", "B", "a", "lx", "lw", "c")}, nx, nu)
                         for t in range(N)])
        self.ring = torch.zeros((self.cap, self.E), **f64)
        self.ring[:N].copy_(torch.as_tensor(host))
        self.start = 0
        self.QxN = torch.as_tensor(np.asarray(prob["QxN"], dtype=np.float64)).to(**f64).contiguous()
        self.lN = torch.as_tensor(np.asarray(prob["lN"], dtype=np.float64)).to(**f64).contiguous()
        self.cN = torch.as_tensor(np.asarray(prob.get("cN", 0.0), dtype=np.float64).reshape(1)).to(**f64)
        self.x0 = torch.as_tensor(np.asarray(prob["x0"], dtype=np.float64)).to(**f64).contiguous()
        self.x = torch.zeros((N + 1, nx), **f64)
        self.w = torch.zeros((N, nu), **f64)
        self.lam = torch.zeros((N + 1, nx), **f64)
        self.obj = torch.zeros(1, **f64)
        self.staging = torch.empty(self.E, dtype=torch.float64, pin_memory=True)
        self.solved = False
        self.busy = False
        self.queue = deque()
        self.t_abs = 0            # absolute index of the window's first stage
        self.current = (0, 0)     # interior leaves whose stored factorization is current
        self.lane = 0

    def footprint(self):
        return 8 * (self.cap * self.E + 2 * (self.N + 1) * self.nx + self.N * self.nu + self.nx * self.nx
                    + 2 * self.nx + 2)

    def shift(self, record, stream):
        """Append one stage record, drop the oldest, x0 <- x_1 of the last
        solution; all copies are queued on `stream`."""
        import torch
        with torch.cuda.stream(stream):
            if self.start + self.N == self.cap:
                # the N - 1 surviving records [N+1, 2N) move to [0, N-1): no overlap
                self.ring[:self.N - 1].copy_(self.ring[self.start + 1:self.start + self.N])
                self.start = -1
            self.staging.numpy()[:] = record
            self.ring[self.start + self.N].copy_(self.staging, non_blocking=True)
            self.start += 1
            self.t_abs += 1
            if self.solved:
                self.x0.copy_(self.x[1])

    def window_host(self):
        r = self.ring[self.start:self.start + self.N].cpu().numpy()
        p = unpack_window(r, self.nx, self.nu, self.N)
        p.update(QxN=self.QxN.cpu().numpy(), lN=self.lN.cpu().numpy(), cN=float(self.cN.cpu()[0]),
                 x0=self.x0.cpu().numpy())
        return p

    def fill_descriptor(self, p):
        nx, nu, N, E = self.nx, self.nu, self.N, self.E
        base = self.ring.data_ptr() + 8 * self.start * E
        offs = record_offsets(nx, nu)
        p.nx, p.nu, p.N = nx, nu, N
        for k in ("Qx", "Qw", "Qxw", "A", "B"):
            setattr(p, k, base + 8 * offs[k])
            setattr(p, "s" + k, E)
        for k in ("a", "lx", "lw", "c"):
            setattr(p, k, base + 8 * offs[k])
            setattr(p, "s" + k, E)
        p.QxN = self.QxN.data_ptr()
        p.x0 = self.x0.data_ptr()
        p.lN = self.lN.data_ptr()
        p.cN = self.cN.data_ptr()
        p.x = self.x.data_ptr()
        p.w = self.w.data_ptr()
        p.lam = self.lam.data_ptr()
        p.obj = self.obj.data_ptr()


class Lane:
    def __init__(self, device):
        import torch
        self.stream = torch.cuda.Stream(device=device)
        self.plan = None
        self.sessions = []        # sessions served by this lane (instance order of its plans)
        self.version = -1
        self.work = None
        self.work_ptr = 0
        self.work_bytes = 0
        self.info = None
        self.probs = None
        self.members = []
        self.event = None
        self.info_host = None     # pinned copy of the status words of the launch in flight
        self.t_launch = 0.0       # host time of the launch in flight
        self.launches = 0
        self.requests = 0
        self.busy_s = 0.0         # launch to retirement, summed


class ServingEngine:
    """Continuous-batching solver for receding-horizon sessions."""

    def __init__(self, precision=rs.RS_FP64, lanes=3, max_batch=1 << 30, hbm_fraction=0.9, tuner=None,
                 device="cuda", record=False, timing=False, record_every=0, rank_reveal=False):
        import torch
        self.torch = torch
        self.device = device
        self.precision = precision
        # rank-revealing master stages let a window's first leaf end at the
        # first leaf boundary (1..Ns stages instead of Ns..2Ns-1), which
        # halves the leaf chain that every request factors again, but every
        # reduction then ends with a pivoted factorization (also on the
        # master levels' critical path); measured, the two cancel for the
        # default sessions, so plain master stages are the default
        self.rank_reveal = rank_reveal
        self.plan_flags = rs.RS_PLAN_RANK_REVEAL if rank_reveal else 0
        self.max_batch = max_batch
        self.tuner = tuner or Tuner()
        free, total = torch.cuda.mem_get_info()
        self.budget = hbm_fraction * total - (total - free)
        self.used = 0
        self.sessions = []
        self.version = 0
        self.lanes = [Lane(device) for _ in range(lanes)]
        self.lat = []
        self.done = 0
        self.failed = 0               # requests whose solve reported a numerical failure
        self.rejected = 0
        self.record = record
        self.record_every = record_every   # > 0: record every k-th served request (a parity sample)
        self.served = 0
        self.results = {}
        self.launches = 0
        self.batch_sizes = []
        self.timing = timing          # per-kernel-kind device time of every launch (HIP events)
        self.kernel_ms = {}
        self.host_s = 0.0             # host time spent preparing launches

    # ------------------------------------------------------------ admission
    def _workspace_per_instance(self, nx, nu, N):
        Ns, br = self.tuner.choose(nx, nu, N, self.precision)
        plan = rs.rs_plan_create_ring([(nx, nu, N, Ns, br, 0, 0, 0)], precision=self.precision,
                                      flags=self.plan_flags)
        try:
            return rs.rs_plan_workspace_size(plan)
        finally:
            rs.rs_plan_destroy(plan)

    def add_session(self, prob):
        """Admit a session if its projected footprint fits; returns its id or None."""
        nx, nu, N = int(prob["QxN"].shape[-1]), int(prob["Qw"].shape[-1]), int(np.shape(prob["lx"])[0])
        try:
            ws = self._workspace_per_instance(nx, nu, N)
        except rs.RsError:          # no kernel for this shape and precision
            self.rejected += 1
            return None
        need = 8 * (2 * N * record_len(nx, nu) + 2 * (N + 1) * nx + N * nu) + ws
        if self.used + need > self.budget:
            self.rejected += 1
            return None
        s = Session(len(self.sessions), prob, self.device)
        # a session always runs on the same lane, whose workspace keeps its
        # stored factorization between requests
        s.lane = self._pick_lane(s)
        self.lanes[s.lane].sessions.append(s)
        self.sessions.append(s)
        self.used += need
        self.version += 1
        return s.sid

    def _pick_lane(self, s):
        """Lane of a new session.  A launch runs its shape groups one after
        another on the lane's stream, and the kernels of a group are chains
        of dependent stages on a few workgroups; lanes that hold one shape
        each run those chains side by side and keep every launch short.  So:
        an empty lane if there is one, else the least loaded lane among
        those that serve this shape only, else the least loaded lane (load =
        sum of N n_x^2, the size of a solve pass)."""
        key = (s.nx, s.nu)
        load = [sum(t.N * t.nx * t.nx for t in lane.sessions) for lane in self.lanes]
        empty = [i for i, lane in enumerate(self.lanes) if not lane.sessions]
        if empty:
            return empty[0]
        same = [i for i, lane in enumerate(self.lanes) if all((t.nx, t.nu) == key for t in lane.sessions)]
        pool = same or range(len(self.lanes))
        return min(pool, key=lambda i: load[i])

    # --------------------------------------------------------------- plans
    def _dims(self, lane):
        """Receding-horizon plan rows of the lane's sessions: window start and
        the interior leaves whose factorization the last request left."""
        rows = []
        for s in lane.sessions:
            Ns, br = self.tuner.choose(s.nx, s.nu, s.N, self.precision)
            rows.append((s.nx, s.nu, s.N, Ns, br, s.t_abs) + tuple(s.current))
        return rows

    def _ensure_workspace(self, lane):
        if lane.version == self.version:
            return
        torch = self.torch
        if lane.plan is not None:
            rs.rs_plan_destroy(lane.plan)
        lane.plan = rs.rs_plan_create_ring(self._dims(lane), precision=self.precision, flags=self.plan_flags)
        lane.work_bytes = rs.rs_plan_workspace_size(lane.plan)
        lane.work = torch.empty(lane.work_bytes + 256, dtype=torch.uint8, device=self.device)
        lane.work_ptr = (lane.work.data_ptr() + 255) // 256 * 256
        lane.info = torch.zeros(2 * len(lane.sessions), dtype=torch.int32, device=self.device)
        lane.info_host = torch.zeros(2 * len(lane.sessions), dtype=torch.int32, pin_memory=True)
        lane.probs = (rs.rs_problem * len(lane.sessions))()
        for i, s in enumerate(lane.sessions):
            s.fill_descriptor(lane.probs[i])
            lane.probs[i].flags = rs.RS_PROB_SKIP
            s.current = (0, 0)         # a new workspace holds no factors yet
        # the status array and the arrays of newly admitted sessions were
        # filled on the current stream; the lane's stream waits for that
        lane.stream.wait_stream(torch.cuda.current_stream())
        lane.version = self.version

    # ------------------------------------------------------------ requests
    def submit(self, sid, record, arrival):
        self.sessions[sid].queue.append((record, arrival))

    def _launch(self, lane, ready):
        torch = self.torch
        h0 = time.perf_counter()
        self._ensure_workspace(lane)
        idx = {id(s): i for i, s in enumerate(lane.sessions)}
        for i in range(len(lane.sessions)):
            lane.probs[i].flags = rs.RS_PROB_SKIP
        lane.members = []
        for s in ready:
            record, arrival = s.queue.popleft()
            s.busy = True
            s.shift(record, lane.stream)
            i = idx[id(s)]
            s.fill_descriptor(lane.probs[i])
            lane.probs[i].flags = 0
            lane.members.append((s, arrival))
        # the lane's receding-horizon plan moved to this launch's windows: the
        # leaves whose stage data the shifts left unchanged keep their stored
        # factorization
        rs.rs_plan_ring_update(lane.plan, self._dims(lane))
        if self.timing:
            rs.rs_plan_set_timing(lane.plan, True)
        rs.rs_batch_solve(lane.plan, lane.probs, lane.work_ptr, lane.work_bytes, lane.stream.cuda_stream,
                          lane.info.data_ptr())
        with torch.cuda.stream(lane.stream):
            lane.info_host.copy_(lane.info, non_blocking=True)
        for s, _ in lane.members:
            Ns, _br = self.tuner.choose(s.nx, s.nu, s.N, self.precision)
            s.current = rs.ring_current_leaves(s.t_abs, s.N, Ns, rank_reveal=self.rank_reveal)
        self.launches += 1
        self.batch_sizes.append(len(ready))
        lane.event = torch.cuda.Event()
        lane.event.record(lane.stream)
        lane.t_launch = h0
        lane.launches += 1
        lane.requests += len(ready)
        self.host_s += time.perf_counter() - h0

    def _complete(self, lane, now):
        if self.timing:
            for k, (ms, n) in rs.rs_plan_kernel_times(lane.plan, reset=True).items():
                if n:
                    self.kernel_ms[k] = self.kernel_ms.get(k, 0.0) + ms
        # the launch's event has completed, so the pinned status copy queued
        # behind the solve on the lane's stream is complete too
        st = lane.info_host.view(-1, 2).numpy()
        idx = {id(s): i for i, s in enumerate(lane.sessions)}
        for s, arrival in lane.members:
            i = idx[id(s)]
            status = int(st[i, 0])
            s.busy = False
            if status == 0:
                s.solved = True
                self.lat.append(now - arrival)
                self.done += 1
            else:
                # a failed solve leaves no usable factors and no x_1: the
                # session's next request factors every leaf again and keeps
                # its initial state
                s.solved = False
                s.current = (0, 0)
                self.failed += 1
            self.served += 1
            if self.record or (self.record_every > 0 and self.served % self.record_every == 0):
                self.results.setdefault(s.sid, []).append(
                    dict(x=s.x.cpu().numpy(), w=s.w.cpu().numpy(), lam=s.lam.cpu().numpy(),
                         obj=float(s.obj.cpu()[0]), status=status, stage=int(st[i, 1]),
                         window=s.window_host()))
        lane.members = []
        lane.event = None
        lane.busy_s += time.perf_counter() - lane.t_launch

    def lane_stats(self):
        """Per lane: shapes, sessions, launches, mean batch and mean time from
        launch to retirement (ms)."""
        out = []
        for lane in self.lanes:
            out.append({"shapes": sorted({"%dx%d" % (t.nx, t.nu) for t in lane.sessions}),
                        "sessions": len(lane.sessions), "launches": lane.launches,
                        "mean_batch": round(lane.requests / lane.launches, 2) if lane.launches else None,
                        "ms_per_launch": round(1e3 * lane.busy_s / lane.launches, 3) if lane.launches else None})
        return out

    def poll(self, now):
        """Retire finished launches, then launch ready sessions on idle lanes."""
        for lane in self.lanes:
            if lane.event is not None and lane.event.query():
                self._complete(lane, now)
        for lane in self.lanes:
            if lane.event is not None:
                continue
            ready = [s for s in lane.sessions if not s.busy and s.queue][:self.max_batch]
            if ready:
                self._launch(lane, ready)

    def busy(self):
        return any(l.event is not None for l in self.lanes) or any(s.queue for s in self.sessions)

    def run(self, trace, log=None):
        """Serve `trace`, a list of (arrival_s, sid, record) sorted by arrival,
        in real time.  Returns summary statistics."""
        t0 = time.perf_counter()
        i, n = 0, len(trace)
        launches0, sizes0 = self.launches, len(self.batch_sizes)
        while i < n or self.busy():
            now = time.perf_counter() - t0
            while i < n and trace[i][0] <= now:
                a, sid, rec = trace[i]
                self.submit(sid, rec, a)
                i += 1
            self.poll(time.perf_counter() - t0)
        el = time.perf_counter() - t0
        sizes = self.batch_sizes[sizes0:]
        lat = np.array(self.lat) * 1e3
        return {"requests": n, "completed": self.done, "failed": self.failed, "elapsed_s": round(el, 3),
                "solves_per_s": round(self.done / el, 1) if el > 0 else None,
                "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
                "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
                "launches": self.launches - launches0,
                "mean_batch": round(float(np.mean(sizes)), 2) if sizes else None,
                "sessions": len(self.sessions), "rejected_sessions": self.rejected,
                "hbm_projected_gb": round(self.used / 1e9, 3), "hbm_budget_gb": round(self.budget / 1e9, 3),
                "host_launch_s": round(self.host_s, 3), "lanes": self.lane_stats(),
                "kernel_ms_total": {k: round(v, 1) for k, v in self.kernel_ms.items()} if self.timing else None}

    def close(self):
        for lane in self.lanes:
            if lane.plan is not None:
                rs.rs_plan_destroy(lane.plan)
                lane.plan = None


# --------------------------------------------------------- synthetic stream
class FixedChoice(Tuner):
    """The same leaf length (raised until the shape allows it) and branch
    for every session."""

    def __init__(self, Ns, branch):
        super().__init__("/nonexistent/fixed-choice.json")
        self.fixed = (Ns, branch if branch > 0 else 4)

    def choose(self, nx, nu, N, precision):
        Ns, br = self.fixed
        while Ns * nu < nx:
            Ns *= 2
        return Ns, br


def poisson_trace(rate, seconds, nsessions, pools, session_shapes, seed):
    """Arrival times of a Poisson process (exponential gaps) with a uniformly
    chosen session per request; the new stage record is drawn from the
    session shape's pool of pre-generated G2 stages."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        sid = int(rng.integers(0, nsessions))
        pool = pools[session_shapes[sid]]
        out.append((t, sid, pool[int(rng.integers(0, len(pool)))]))
    return out


def stage_pool(nx, nu, count, seed):
    from . import workloads as W
    p = W.g2(nx, nu, count, seed=seed)
    return [pack_stage({k: p[k][t] for k in ("Qx", "Qw", "Qxw", "A", "B", "a", "lx", "lw", "c")}, nx, nu)
            for t in range(count)]


def main(argv=None):
    import argparse
    import json
    from . import workloads as W
    ap = argparse.ArgumentParser(description="Receding-horizon serving benchmark (one GPU)")
    ap.add_argument("--rate", type=float, default=5000.0)
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--warmup-seconds", type=float, default=1.0)
    ap.add_argument("--sessions", type=int, default=64)
    ap.add_argument("--nx", default="8,32,64", help="state dimensions; n_u = n_x / 2")
    ap.add_argument("--Nmin", type=int, default=64)
    ap.add_argument("--Nmax", type=int, default=4096)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed")
    ap.add_argument("--lanes", type=int, default=3)
    ap.add_argument("--rank-reveal", action="store_true",
                    help="rank-revealing master stages (a window's first leaf then ends at the first boundary)")
    ap.add_argument("--seed", type=int, default=W.seed_for(3))
    ap.add_argument("--timing", action="store_true", help="report device time per kernel kind")
    ap.add_argument("--Ns", type=int, default=32, help="leaf length for every session (0: the tuner's choice)")
    ap.add_argument("--branch", type=int, default=8, help="master branch for every session (0: the tuner's)")
    args = ap.parse_args(argv)
    import torch
    rng = np.random.default_rng(args.seed)
    nxs = [int(v) for v in args.nx.split(",")]
    prec = rs.RS_FP64 if args.precision == "fp64" else rs.RS_MIXED_FP32
    tuner = FixedChoice(args.Ns, args.branch) if args.Ns > 0 else None
    eng = ServingEngine(precision=prec, lanes=args.lanes, timing=args.timing, tuner=tuner,
                        rank_reveal=args.rank_reveal)
    shapes = []
    for i in range(args.sessions):
        nx = nxs[int(rng.integers(0, len(nxs)))]
        N = int(rng.integers(args.Nmin, args.Nmax + 1))
        sid = eng.add_session(W.g2(nx, nx // 2, N, seed=args.seed + 17 * i))
        if sid is not None:
            shapes.append((nx, nx // 2))
    print("serving: %d sessions admitted (%s)" % (len(shapes), ", ".join(sorted(set("%dx%d" % s for s in shapes)))),
          file=sys.stderr, flush=True)
    pools = {sh: stage_pool(sh[0], sh[1], 64, seed=args.seed + sh[0]) for sh in set(shapes)}
    warm = poisson_trace(args.rate, args.warmup_seconds, len(shapes), pools, shapes, args.seed + 1)
    eng.run(warm)
    torch.cuda.synchronize()
    eng.lat, eng.done, eng.failed, eng.kernel_ms, eng.host_s = [], 0, 0, {}, 0.0
    for lane in eng.lanes:
        lane.launches, lane.requests, lane.busy_s = 0, 0, 0.0
    trace = poisson_trace(args.rate, args.seconds, len(shapes), pools, shapes, args.seed + 2)
    out = eng.run(trace)
    out.update({"rate_req_s": args.rate, "precision": args.precision,
                "shapes": sorted(set("%dx%d" % s for s in shapes)), "N_range": [args.Nmin, args.Nmax]})
    print(json.dumps(out), flush=True)
    eng.close()


if __name__ == "__main__":
    main()
