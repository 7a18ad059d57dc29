"""ctypes front end of the sequential FP64 oracle (ks_oracle.c).

TEST INFRASTRUCTURE: see the package docstring.  Inputs are numpy arrays in the
step-major layout documented in ks_oracle.h; any object with the attributes
k, n, m, H, F, c, K, G, o, C, K_diag, C_diag can be passed to ``smooth``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

OK, E_ARG, E_NOT_SPD, E_RANK, E_NOMEM = 0, -1, -3, -4, -9

_lib = None


def load(path: str | None = None):
    global _lib
    if path is not None:
        lib = ctypes.CDLL(path)
    else:
        if _lib is not None:
            return _lib
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("kso_smooth", "kso_smooth_rts"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      ctypes.c_int] + [dp] * 7 + [dp] * 4
    if path is None:
        _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def smooth(p, want_cov: bool = True, want_lag1: bool = False, lib=None, check: bool = True,
           rts: bool = False):
    """Run the sequential oracle on problem ``p``.

    Returns a dict with 'u' [k+1][n], 'cov' [k+1][n][n] (or None), 'lag1'
    [k][n][n] (or None), 'resid2' and 'status'.  Covariances come from the RTS
    recursion in square-root information form over the QR factor R, or, with
    rts=True, from the RTS recursion in information form over the model
    matrices (the cross-check; its error grows with the condition number of
    the normal matrix).
    """
    lib = lib or load()
    k, n, m = int(p.k), int(p.n), int(p.m)
    arrs = [_c64(a) for a in (p.H, p.F, p.c, p.K, p.G, p.o, p.C)]
    u = np.zeros((k + 1, n))
    cov = np.zeros((k + 1, n, n)) if want_cov else None
    lag1 = np.zeros((max(k, 0), n, n)) if want_lag1 else None
    r2 = np.zeros(1)
    fn = lib.kso_smooth_rts if rts else lib.kso_smooth
    st = fn(k, n, m, int(bool(p.K_diag)), int(bool(p.C_diag)),
                        *[_ptr(a) for a in arrs], _ptr(u), _ptr(cov), _ptr(lag1), _ptr(r2))
    if check and st != OK:
        raise OracleError(st)
    return dict(u=u, cov=cov, lag1=lag1, resid2=float(r2[0]), status=st)
