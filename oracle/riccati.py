"""ctypes front-end of the serial FP64 Riccati oracle (paper Sec. 3, Alg. 1-3).

Test infrastructure only (see the package docstring).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def use_library(path):
    """Load the oracle from another build of the same source (the host-tuned
    build the timed CPU baseline uses); the next call loads it."""
    global _lib, _path
    _lib, _path = None, path


# ORACLE_LIBRARY names another build of the same source (the sanitized copy
# that the sanitizer test loads)
_path = os.environ.get("ORACLE_LIBRARY")


def _load():
    global _lib
    if _lib is None:
        path = _path or _build.ensure_built()
        lib = ctypes.CDLL(path)
        dp = ctypes.c_void_p
        lib.oracle_riccati_solve.restype = ctypes.c_int
        lib.oracle_riccati_solve.argtypes = (
            [ctypes.c_int] * 3 + [dp] * 11 + [ctypes.c_double] + [dp] * 11)
        _lib = lib
    return _lib


def _ptr(arr):
    return None if arr is None else arr.ctypes.data


def _f64(arr):
    return None if arr is None else np.ascontiguousarray(arr, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def solve(prob, want_factors=False):
    """Solve the UFTOC problem P(N) by Alg. 1-3.

    Returns a dict with ``x (N+1,nx)``, ``w (N,nu)``, ``lam (N+1,nx)``,
    ``obj`` (optimal value) and, if ``want_factors``, ``P (N+1,nx,nx)``,
    ``Psi (N+1,nx)``, ``cbar (N+1,)``, ``K (N,nu,nx)``, ``k (N,nu)`` and
    ``G (N,nu,nu)`` where block t holds the quantity the paper indexes t+1
    for K, k and G (the ones used at stage t).

    Raises ``OracleError`` if some G_{t+1} is not positive definite.
    """
    lib = _load()
    Qx, Qw, A, B = (_f64(prob[k]) for k in ("Qx", "Qw", "A", "B"))
    N, nx, nu = Qx.shape[0], prob["QxN"].shape[0], Qw.shape[1]
    Qxw = _f64(prob.get("Qxw"))
    a, lx, lw, c = (_f64(prob.get(k)) for k in ("a", "lx", "lw", "c"))
    QxN, lN, x0 = _f64(prob["QxN"]), _f64(prob.get("lN")), _f64(prob["x0"])
    cN = float(prob.get("cN", 0.0))
    x = np.zeros((N + 1, nx))
    w = np.zeros((N, nu))
    lam = np.zeros((N + 1, nx))
    obj = np.zeros(1)
    if want_factors:
        P = np.zeros((N + 1, nx, nx))
        Psi = np.zeros((N + 1, nx))
        cbar = np.zeros(N + 1)
        K = np.zeros((N, nu, nx))
        k = np.zeros((N, nu))
        G = np.zeros((N, nu, nu))
    else:
        P = Psi = cbar = K = k = G = None
    st = lib.oracle_riccati_solve(
        nx, nu, N, _ptr(Qx), _ptr(Qw), _ptr(Qxw), _ptr(A), _ptr(B), _ptr(a),
        _ptr(lx), _ptr(lw), _ptr(c), _ptr(QxN), _ptr(lN), cN, _ptr(x0),
        _ptr(x), _ptr(w), _ptr(lam), _ptr(obj), _ptr(P), _ptr(Psi), _ptr(cbar),
        _ptr(K), _ptr(k), _ptr(G))
    if st != 0:
        if st == -1000000:
            raise MemoryError("oracle: allocation failed")
        raise OracleError("G_{t+1} not positive definite at stage t=%d" % (-st - 1))
    out = dict(x=x, w=w, lam=lam, obj=float(obj[0]))
    if want_factors:
        out.update(P=P, Psi=Psi, cbar=cbar, K=K, k=k, G=G)
    return out
