"""Exact covariance-vector product y = C w for large n (Section 1, eq. (2)
with the nugget on the diagonal) -- TEST INFRASTRUCTURE ONLY.

C is never formed: oracle/matvec.c evaluates each entry on the fly (O(n^2)
work, O(n) memory), so at n = 256,000, where the dense matrix would need
488 GiB, it still gives the exact product. Only nu = 1/2 and nu = 3/2, the
smoothness values with an elementary closed form, are offered. With
Z = C w the quadratic form of eq. (1) is known exactly, Z^T C^{-1} Z = w^T Z,
which pins the H-matrix solve at any size.

The C file is compiled with gcc on first use into oracle/_build (or by the
package's build step) and loaded with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "matvec.c")
LIB = os.path.join(HERE, "_build", "liboracle_matvec.so")

_lib = None


def build() -> str:
    """Compile matvec.c (gcc, OpenMP) into oracle/_build."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + f".{os.getpid()}.tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.oracle_cov_matvec.restype = ctypes.c_int
        L.oracle_cov_matvec.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                        ctypes.c_long, ctypes.c_void_p]
        _lib = L
    return _lib


def cov_matvec(pts, theta, w) -> np.ndarray:
    """C(theta) w for points pts (n, d), theta = (sigma2, ell, nu, tau2) with nu in
    {0.5, 1.5}; w of shape (n,) or (n, k) with k <= 16 (one pass over the entries)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    vec = w.ndim == 1
    W = np.ascontiguousarray(w.reshape(w.shape[0], -1))
    n, dim = pts.shape
    if W.shape[0] != n or W.shape[1] > 16:
        raise ValueError("w must have n rows and at most 16 columns")
    sigma2, ell, nu, tau2 = (float(v) for v in theta)
    if nu not in (0.5, 1.5):
        raise ValueError("the exact product covers nu = 1/2 and nu = 3/2 only")
    Y = np.empty_like(W)
    st = _load().oracle_cov_matvec(pts.ctypes.data, n, dim, sigma2, ell, int(round(2 * nu)), tau2, W.ctypes.data,
                                   W.shape[1], Y.ctypes.data)
    if st != 0:
        raise ValueError("bad arguments")
    return Y[:, 0] if vec else Y
