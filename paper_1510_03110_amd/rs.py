"""Python binding of the C ABI in ``include/rs.h`` (ctypes; argument
marshalling only - every step of the solve runs in the HIP library).

The entry points keep the C names: ``rs_plan_create``,
``rs_plan_workspace_size``, ``rs_plan_destroy``, ``rs_batch_solve``,
``rs_factor``, ``rs_solve``, ``rs_plan_query``, ``rs_plan_export``,
``rs_status_string``.  ``Batch`` packs stacked torch device tensors into the
descriptor array the library expects.  PyTorch provides device memory and
streams only.
"""
import ctypes
import os

import numpy as np

from . import build as _build

RS_OK, RS_ERR_ARG, RS_ERR_NOT_SPD, RS_ERR_SINGULAR_MASTER, RS_ERR_NOT_CONVERGED, \
    RS_ERR_NOMEM, RS_ERR_HIP, RS_ERR_UNSUPPORTED = range(8)
RS_FP64, RS_MIXED_FP32, RS_MIXED_BF16 = 0, 1, 2
RS_PLAN_FACTORED = 1
RS_PLAN_RANK_REVEAL = 2
RS_PLAN_REPORT = 4
RS_PLAN_CHECK_INPUTS = 8
RS_PLAN_NATIVE_TILES = 16
RS_PLAN_REFACTOR_DOWN = 32
RS_PROB_SKIP = 1
RS_KERNEL_KINDS = 16

_P = ctypes.c_void_p


class rs_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nu", ctypes.c_int32), ("N", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("Qx", _P), ("sQx", ctypes.c_int64), ("Qw", _P), ("sQw", ctypes.c_int64),
                ("Qxw", _P), ("sQxw", ctypes.c_int64), ("A", _P), ("sA", ctypes.c_int64),
                ("B", _P), ("sB", ctypes.c_int64), ("QxN", _P),
                ("x0", _P), ("a", _P), ("lx", _P), ("lw", _P), ("c", _P), ("lN", _P), ("cN", _P),
                ("x", _P), ("w", _P), ("lam", _P), ("obj", _P),
                ("sa", ctypes.c_int64), ("slx", ctypes.c_int64), ("slw", ctypes.c_int64), ("sc", ctypes.c_int64)]


class rs_mhe(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("Nmhe", ctypes.c_int32),
                ("nw", ctypes.c_int32)] + \
               [f for k in ("A", "B", "a", "C", "d", "y", "wtil", "vtil", "Qw", "Qv", "Qwv")
                for f in ((k, _P), ("s" + k, ctypes.c_int64))] + \
               [("xtil0", _P), ("Ptil0", _P)]


class rs_ip(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nu", ctypes.c_int32), ("N", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("prob", rs_problem), ("wlo", _P), ("swlo", ctypes.c_int64), ("whi", _P), ("swhi", ctypes.c_int64),
                ("ml", _P), ("mu", _P), ("newton", rs_problem), ("dw_aff", _P), ("dml", _P), ("dmu", _P),
                ("part", _P), ("stats", _P)]


class rs_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("Ns", ctypes.c_int32), ("branch", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("tol", ctypes.c_double), ("flags", ctypes.c_int32),
                ("leaf_chunk", ctypes.c_int32)]


class rs_info(ctypes.Structure):
    _fields_ = [("rel_resid", ctypes.c_double), ("bwd_err", ctypes.c_double), ("est_fwd_err", ctypes.c_double),
                ("refine_iters", ctypes.c_int32), ("bad_stage", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RsError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, rs_status_string(status), status))


_lib = None


def library():
    """Load ``librs.so`` (building it first only if no build exists).
    RS_LIBRARY names another build of the same sources (the host-sanitized
    copy that the sanitizer test loads)."""
    global _lib
    if _lib is None:
        path = os.environ.get("RS_LIBRARY") or _build.LIB_PATH
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        lib.rs_plan_create.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(rs_options), ctypes.POINTER(_P)]
        lib.rs_plan_create_ex.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(rs_options), ctypes.POINTER(_P)]
        lib.rs_plan_create_split.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                             ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(rs_options),
                                             ctypes.POINTER(_P)]
        lib.rs_plan_create_ring.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(rs_options), ctypes.POINTER(_P)]
        lib.rs_plan_ring_update.argtypes = [_P, ctypes.POINTER(i32)]
        lib.rs_mhe_to_uftoc.argtypes = [i32, ctypes.POINTER(rs_mhe), ctypes.POINTER(rs_problem), _P, _P]
        lib.rs_mhe_to_uftoc.restype = i32
        for name, extra in (("rs_ip_newton", [i32, ctypes.c_double]), ("rs_ip_step", [i32, ctypes.c_double]),
                            ("rs_ip_mu", [ctypes.c_double, ctypes.c_double]),
                            ("rs_ip_update", [ctypes.c_double, ctypes.c_double])):
            getattr(lib, name).argtypes = [ctypes.POINTER(rs_ip)] + extra + [_P]
            getattr(lib, name).restype = i32
        lib.rs_graph_create.argtypes = [_P, i32, ctypes.POINTER(rs_problem), _P, sz, _P, _P, ctypes.POINTER(_P)]
        lib.rs_graph_launch.argtypes = [_P, _P]
        lib.rs_graph_destroy.argtypes = [_P]
        lib.rs_plan_workspace_size.argtypes = [_P, ctypes.POINTER(sz)]
        lib.rs_plan_destroy.argtypes = [_P]
        for name in ("rs_batch_solve", "rs_factor", "rs_solve"):
            getattr(lib, name).argtypes = [_P, ctypes.POINTER(rs_problem), _P, sz, _P, _P]
        lib.rs_plan_query.argtypes = [_P, i32]
        lib.rs_plan_query.restype = i64
        lib.rs_plan_export.argtypes = [_P, i32, ctypes.POINTER(i64), i64]
        lib.rs_plan_export.restype = i64
        lib.rs_plan_set_timing.argtypes = [_P, i32]
        lib.rs_plan_set_timing.restype = i32
        lib.rs_plan_kernel_times.argtypes = [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]
        lib.rs_plan_kernel_times.restype = i32
        lib.rs_refine_stats.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_double), _P]
        lib.rs_refine_stats.restype = i32
        lib.rs_info_report.argtypes = [_P, _P, _P, _P, _P]
        lib.rs_info_report.restype = i32
        lib.rs_batch_solve_noalloc.argtypes = [_P, ctypes.POINTER(rs_problem), _P, _P]
        lib.rs_batch_solve_noalloc.restype = i32
        lib.rs_status_string.argtypes = [i32]
        lib.rs_status_string.restype = ctypes.c_char_p
        for name in ("rs_plan_create", "rs_plan_create_ex", "rs_plan_create_split", "rs_plan_create_ring",
                     "rs_plan_ring_update",
                     "rs_plan_workspace_size",
                     "rs_plan_destroy",
                     "rs_batch_solve", "rs_factor", "rs_solve", "rs_graph_create", "rs_graph_launch",
                     "rs_graph_destroy"):
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


def rs_status_string(status):
    return library().rs_status_string(int(status)).decode()


def _check(status, where):
    if status != RS_OK:
        raise RsError(status, where)


def rs_plan_create_split(dims, leaf_lens, branches, precision=RS_FP64, max_refine=0, tol=0.0, flags=0):
    """dims: sequence of (nx, nu, N); leaf_lens[i]: the leaf lengths of
    instance i in stage order (summing to N); branches[i]: its master group
    sizes for levels 1, 2, ... (the last repeats)."""
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
    P32 = ctypes.POINTER(ctypes.c_int32)
    lo = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(v) for v in leaf_lens])]).astype(np.int32))
    ll = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.int32) for v in leaf_lens]).astype(np.int32))
    bo = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(v) for v in branches])]).astype(np.int32))
    bb = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.int32) for v in branches]).astype(np.int32))
    opt = rs_options(precision, 0, 0, max_refine, tol, flags, 0)
    h = _P()
    st = library().rs_plan_create_split(d.shape[0], d.ctypes.data_as(P32), lo.ctypes.data_as(P32),
                                        ll.ctypes.data_as(P32), bo.ctypes.data_as(P32), bb.ctypes.data_as(P32),
                                        ctypes.byref(opt), ctypes.byref(h))
    _check(st, "rs_plan_create_split")
    return h


def rs_plan_create(dims, precision=RS_FP64, Ns=0, branch=0, max_refine=0, tol=0.0, flags=0, leaf_chunk=0):
    """dims: sequence of (nx, nu, N), or of (nx, nu, N, Ns, branch) for a
    leaf length and branch per instance (rs_plan_create_ex).  Returns an
    opaque plan handle."""
    arr = np.asarray(dims, dtype=np.int32)
    width = 5 if arr.ndim == 2 and arr.shape[1] == 5 else 3
    arr = np.ascontiguousarray(arr.reshape(-1, width))
    opt = rs_options(precision, Ns, branch, max_refine, tol, flags, leaf_chunk)
    h = _P()
    fn = library().rs_plan_create_ex if width == 5 else library().rs_plan_create
    st = fn(arr.shape[0], arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(opt), ctypes.byref(h))
    _check(st, "rs_plan_create")
    return h


def rs_plan_create_ring(dims8, precision=RS_FP64, max_refine=0, tol=0.0, flags=0):
    """Receding-horizon plan: dims8 rows (nx, nu, N, Ns, branch, start,
    reuse_lo, reuse_hi); see ring_current_leaves for the reuse range a call
    leaves behind."""
    arr = np.ascontiguousarray(np.asarray(dims8, dtype=np.int32).reshape(-1, 8))
    opt = rs_options(precision, 0, 0, max_refine, tol, flags, 0)
    h = _P()
    st = library().rs_plan_create_ring(arr.shape[0], arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       ctypes.byref(opt), ctypes.byref(h))
    _check(st, "rs_plan_create_ring")
    return h


def rs_plan_ring_update(plan, dims8):
    """New window positions / reuse ranges for a receding-horizon plan."""
    arr = np.ascontiguousarray(np.asarray(dims8, dtype=np.int32).reshape(-1, 8))
    _check(library().rs_plan_ring_update(plan, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "rs_plan_ring_update")


def rs_mhe_to_uftoc(mhe, probs, stream_ptr=None, info_ptr=None):
    """Device MHE -> UFTOC conversion; mhe, probs: ctypes arrays of equal length."""
    _check(library().rs_mhe_to_uftoc(len(mhe), mhe, probs, stream_ptr, info_ptr), "rs_mhe_to_uftoc")


def ring_current_leaves(start, N, Ns, rank_reveal=False):
    """Absolute interior leaves [lo, hi) whose stored factorization a
    receding-horizon call with window start `start` leaves current (plans
    with RS_PLAN_RANK_REVEAL end the first leaf at the first boundary)."""
    first_end = (start // Ns + (1 if (start % Ns == 0 or rank_reveal) else 2)) * Ns
    if start + N <= first_end:
        return 0, 0
    return first_end // Ns, (start + N - 1) // Ns


def rs_plan_workspace_size(plan):
    n = ctypes.c_size_t()
    _check(library().rs_plan_workspace_size(plan, ctypes.byref(n)), "rs_plan_workspace_size")
    return n.value


def rs_plan_destroy(plan):
    _check(library().rs_plan_destroy(plan), "rs_plan_destroy")


def rs_plan_query(plan, key):
    return int(library().rs_plan_query(plan, key))


def rs_plan_export(plan, what):
    lib = library()
    rows = lib.rs_plan_export(plan, what, None, 0)
    width = 7 if what == 0 else 11
    out = np.zeros((max(rows, 1), width), dtype=np.int64)
    lib.rs_plan_export(plan, what, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows)
    return out[:rows]


KERNEL_KINDS = ("init", "leaf_up", "tree", "leaf_down", "factor_leaf_up", "factor_tree", "factor_leaf_down",
                "solve_leaf_up", "solve_tree", "solve_leaf_down", "residual", "update", "check")


def rs_plan_set_timing(plan, enable):
    _check(library().rs_plan_set_timing(plan, int(bool(enable))), "rs_plan_set_timing")


def rs_plan_kernel_times(plan, reset=True):
    """{kind: (total_ms, launches)} since the last reset (synchronizes)."""
    ms = (ctypes.c_double * RS_KERNEL_KINDS)()
    n = (ctypes.c_int64 * RS_KERNEL_KINDS)()
    _check(library().rs_plan_kernel_times(plan, ms, n, int(bool(reset))), "rs_plan_kernel_times")
    return {KERNEL_KINDS[k]: (ms[k], n[k]) for k in range(len(KERNEL_KINDS))}


REFINE_STATS = ("rel_residual", "est_forward_error", "corrections", "converged", "last_correction")


def rs_refine_stats(plan, work_ptr, count, stream_ptr=None):
    """(count, 5) array, columns REFINE_STATS (synchronizes the stream)."""
    out = np.zeros(5 * count, dtype=np.float64)
    _check(library().rs_refine_stats(plan, work_ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     stream_ptr), "rs_refine_stats")
    return out.reshape(count, 5)


def rs_info_report(plan, work_ptr, info_ptr, report_ptr, stream_ptr=None):
    """Queue the per-instance rs_info records of the last solve into the
    device buffer at report_ptr (40 bytes per instance)."""
    _check(library().rs_info_report(plan, work_ptr, info_ptr, report_ptr, stream_ptr), "rs_info_report")


RS_INFO_DTYPE = np.dtype([("rel_resid", "<f8"), ("bwd_err", "<f8"), ("est_fwd_err", "<f8"),
                          ("refine_iters", "<i4"), ("bad_stage", "<i4"), ("status", "<i4"), ("reserved", "<i4")])


def _call(name, plan, probs, work_ptr, work_bytes, stream_ptr, info_ptr):
    st = getattr(library(), name)(plan, probs, work_ptr, work_bytes, stream_ptr, info_ptr)
    _check(st, name)


def rs_batch_solve(plan, probs, work_ptr, work_bytes, stream_ptr=None, info_ptr=None):
    _call("rs_batch_solve", plan, probs, work_ptr, work_bytes, stream_ptr, info_ptr)


def rs_batch_solve_noalloc(plan, probs, stream_ptr=None, info_ptr=None):
    """rs_batch_solve on the library's static device scratch (no workspace)."""
    _check(library().rs_batch_solve_noalloc(plan, probs, stream_ptr, info_ptr), "rs_batch_solve_noalloc")


RS_NOALLOC_SCRATCH_BYTES = 64 << 20


def rs_factor(plan, probs, work_ptr, work_bytes, stream_ptr=None, info_ptr=None):
    _call("rs_factor", plan, probs, work_ptr, work_bytes, stream_ptr, info_ptr)


def rs_solve(plan, probs, work_ptr, work_bytes, stream_ptr=None, info_ptr=None):
    _call("rs_solve", plan, probs, work_ptr, work_bytes, stream_ptr, info_ptr)


def rs_graph_create(plan, mode, probs, work_ptr, work_bytes, stream_ptr, info_ptr=None):
    """Capture one call (0 batch solve, 1 factor, 2 solve) into a HIP graph."""
    h = _P()
    _check(library().rs_graph_create(plan, mode, probs, work_ptr, work_bytes, stream_ptr, info_ptr,
                                     ctypes.byref(h)), "rs_graph_create")
    return h


def rs_graph_launch(graph, stream_ptr):
    _check(library().rs_graph_launch(graph, stream_ptr), "rs_graph_launch")


def rs_graph_destroy(graph):
    _check(library().rs_graph_destroy(graph), "rs_graph_destroy")


# ------------------------------------------------------------ torch helper
_MATS = ("Qx", "Qw", "Qxw", "A", "B")
_VECS = ("a", "lx", "lw", "c", "lN", "cN", "x0")


class Batch:
    """A batch of problems held in torch device tensors plus its plan and
    workspace.

    ``data`` maps the problem keys to tensors with a leading instance axis
    (uniform shapes) or to lists of per-instance tensors (shapes may differ).
    Outputs ``x``, ``w``, ``lam``, ``obj`` are allocated here.  Time-invariant
    matrices may be given with a stage axis of length 1; they are passed with
    stride 0.  ``factored=True`` reserves the stored factorization so that
    ``factor()`` / ``solve_factored()`` can be used.  ``rank_reveal=True``
    gives the master problems rank-revealing stages (RS_PLAN_RANK_REVEAL), so
    that leaves with Ns * nu < nx, or whose inputs leave state directions
    unreached, are allowed.  ``split=(leaf_lens, branches)`` gives every
    instance its own leaf lengths and per-level master group sizes
    (rs_plan_create_split).  ``report=True`` sets RS_PLAN_REPORT (per-instance
    residual, backward error and forward-error estimate, read by ``report()``).
    """

    def __init__(self, data, precision=RS_FP64, Ns=0, branch=0, max_refine=0, tol=0.0,
                 device="cuda", factored=False, per_instance=None, rank_reveal=False, split=None, report=False,
                 leaf_chunk=0, check_inputs=False, flags=0):
        import torch
        self.torch = torch
        keys = set(data)
        self.count = len(data["x0"])
        self.data = {}
        for k in keys:
            v = data[k]
            if isinstance(v, (list, tuple)):
                self.data[k] = [self._dev(t, device) for t in v]
            else:
                self.data[k] = [self._dev(v[i], device) for i in range(self.count)]
        dims = []
        for i in range(self.count):
            nx = int(self.data["QxN"][i].shape[-1])
            nu = int(self.data["Qw"][i].shape[-1])
            N = int(self.data["N"][i]) if "N" in self.data else int(self.data["lx"][i].shape[0])
            dims.append((nx, nu, N))
        self.dims = dims
        f64 = dict(dtype=torch.float64, device=device)
        self.x = [torch.zeros((N + 1, nx), **f64) for nx, nu, N in dims]
        self.w = [torch.zeros((N, nu), **f64) for nx, nu, N in dims]
        self.lam = [torch.zeros((N + 1, nx), **f64) for nx, nu, N in dims]
        self.obj = torch.zeros(self.count, **f64)
        self.info = torch.zeros(2 * self.count, dtype=torch.int32, device=device)
        pdims = dims if per_instance is None else [d + tuple(pi) for d, pi in zip(dims, per_instance)]
        flags = (RS_PLAN_FACTORED if factored else 0) | (RS_PLAN_RANK_REVEAL if rank_reveal else 0) | \
            (RS_PLAN_REPORT if report else 0) | (RS_PLAN_CHECK_INPUTS if check_inputs else 0) | int(flags)
        if split is not None:
            self.plan = rs_plan_create_split(dims, split[0], split[1], precision, max_refine, tol, flags)
        else:
            self.plan = rs_plan_create(pdims, precision, Ns, branch, max_refine, tol, flags, leaf_chunk)
        self.graphs = []
        self.work_bytes = rs_plan_workspace_size(self.plan)
        self.work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device=device)
        base = self.work.data_ptr()
        self.work_ptr = (base + 255) // 256 * 256
        self.probs = (rs_problem * self.count)()
        self._fill()

    @staticmethod
    def _dev(t, device):
        import torch
        if isinstance(t, np.ndarray) or np.isscalar(t):
            t = torch.as_tensor(np.asarray(t, dtype=np.float64))
        return t.to(device=device, dtype=torch.float64).contiguous()

    def _fill(self):
        for i, (nx, nu, N) in enumerate(self.dims):
            p = self.probs[i]
            d = {k: self.data[k][i] for k in self.data}
            p.nx, p.nu, p.N = nx, nu, N
            for k, bs in (("Qx", nx * nx), ("Qw", nu * nu), ("Qxw", nx * nu), ("A", nx * nx), ("B", nx * nu)):
                t = d.get(k)
                if t is None:
                    setattr(p, k, None)
                    setattr(p, "s" + k, 0)
                    continue
                setattr(p, k, t.data_ptr())
                stride = 0 if (t.dim() == 3 and t.shape[0] == 1 and N > 1) else bs
                setattr(p, "s" + k, stride)
            p.QxN = d["QxN"].data_ptr()
            for k in _VECS:
                t = d.get(k)
                setattr(p, k, t.data_ptr() if t is not None else None)
            # stage vectors: dense, or one vector for every stage (stage axis 1)
            for k, bs in (("a", nx), ("lx", nx), ("lw", nu), ("c", 1)):
                t = d.get(k)
                one = t is not None and t.numel() == bs and N > 1
                setattr(p, "s" + k, 0 if one else bs)
            p.x = self.x[i].data_ptr()
            p.w = self.w[i].data_ptr()
            p.lam = self.lam[i].data_ptr()
            p.obj = self.obj.data_ptr() + 8 * i

    def stream_ptr(self):
        return self.torch.cuda.current_stream().cuda_stream

    def solve(self):
        rs_batch_solve(self.plan, self.probs, self.work_ptr, self.work_bytes, self.stream_ptr(),
                       self.info.data_ptr())

    def factor(self):
        rs_factor(self.plan, self.probs, self.work_ptr, self.work_bytes, self.stream_ptr(),
                  self.info.data_ptr())

    def solve_factored(self):
        rs_solve(self.plan, self.probs, self.work_ptr, self.work_bytes, self.stream_ptr(),
                 self.info.data_ptr())

    def set_skip(self, i, skip=True):
        """Exclude instance i from the following calls (RS_PROB_SKIP)."""
        self.probs[i].flags = RS_PROB_SKIP if skip else 0

    def refine_stats(self):
        return rs_refine_stats(self.plan, self.work_ptr, self.count, self.stream_ptr())

    def report(self):
        """Per-instance rs_info records of the last solve (numpy structured
        array with the fields of rs_info; synchronizes)."""
        torch = self.torch
        buf = torch.zeros(40 * self.count, dtype=torch.uint8, device=self.info.device)
        rs_info_report(self.plan, self.work_ptr, self.info.data_ptr(), buf.data_ptr(), self.stream_ptr())
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=RS_INFO_DTYPE)

    def update(self, key, i, values):
        """Overwrite problem field ``key`` of instance ``i`` in place (same
        device buffer, so the descriptors stay valid)."""
        t = self.data[key][i]
        t.copy_(self._dev(values, t.device).reshape(t.shape))

    def capture(self, mode=0):
        """HIP graph of solve (0), factor (1) or solve_factored (2) on a side
        stream; replay it with ``replay``."""
        torch = self.torch
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = rs_graph_create(self.plan, mode, self.probs, self.work_ptr, self.work_bytes, side.cuda_stream,
                            self.info.data_ptr())
        torch.cuda.current_stream().wait_stream(side)
        self.graphs.append(g)
        return g

    def replay(self, graph):
        rs_graph_launch(graph, self.stream_ptr())

    def status(self):
        return self.info.view(-1, 2).cpu().numpy()

    def result(self, i):
        return dict(x=self.x[i].cpu().numpy(), w=self.w[i].cpu().numpy(),
                    lam=self.lam[i].cpu().numpy(), obj=float(self.obj[i].cpu()))

    def close(self):
        for g in getattr(self, "graphs", []):
            rs_graph_destroy(g)
        self.graphs = []
        if self.plan is not None:
            rs_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
