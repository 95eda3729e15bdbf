"""Test infrastructure only: the FP64 CPU oracle for the GLS grid.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package; the GPU product path never does.

`gls` wraps the plain C oracle (oracle.c): for each (SNP, trait) problem it
solves Eq. (1) of the paper, b = (X^T M^{-1} X)^{-1} X^T M^{-1} y, with the
covariance of Eq. (2), M = sigma2 (h2 Phi + (1 - h2) I), through a dense
Cholesky factorisation of M (Section 3.1), in O(n^3) per trait.

`rotated` (rotated.py) is a second, independent CPU reference: Eq. (1) with
M_j^{-1} = Z diag(d_j) Z^T from the eigendecomposition of Phi (Section 3.1),
each problem's p x p normal equations formed in the rotated basis, in numpy FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP) into liboracle.so, in place."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_gls.restype = ctypes.c_int
        lib.oracle_gls.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, dp,
                                   ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int32), dp,
                                   ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gls(phi, xl, xr_cols, y, h2, trait=None, sigma2=None, nthreads: int = 0,
        return_non_spd: bool = False):
    """Solve one GLS problem per row of xr_cols.

    phi      [n][n] kinship (symmetric)
    xl       [(p-1)][n] covariate columns X_L
    xr_cols  [q][n] the SNP column x_i of each problem
    y        [T][n] traits; h2 [T]; sigma2 [T] or None (ones)
    trait    [q] trait index of each problem (default: problem q uses trait q)
    Returns b [q][p] FP64 (NaN where X_i^T M^{-1} X_i is not SPD).
    """
    lib = _load()
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    xl = np.ascontiguousarray(np.atleast_2d(xl), dtype=np.float64)
    xr = np.ascontiguousarray(np.atleast_2d(xr_cols), dtype=np.float64)
    y = np.ascontiguousarray(np.atleast_2d(y), dtype=np.float64)
    h2 = np.ascontiguousarray(np.atleast_1d(h2), dtype=np.float64)
    n = phi.shape[0]
    p = xl.shape[0] + 1
    q = xr.shape[0]
    if trait is None:
        trait = np.arange(q)
    trait = np.ascontiguousarray(trait, dtype=np.int32)
    if phi.shape != (n, n) or xl.shape[1] != n or xr.shape[1] != n or y.shape[1] != n \
            or h2.shape[0] != y.shape[0] or trait.shape[0] != q:
        raise ValueError("inconsistent shapes")
    sg = None
    if sigma2 is not None:
        sg = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
        if sg.shape[0] != y.shape[0]:
            raise ValueError("sigma2 needs one value per trait")
    b = np.empty((q, p))
    bad = ctypes.c_int64(0)
    rc = lib.oracle_gls(n, p, _dp(phi), _dp(xl), y.shape[0], _dp(y), _dp(h2),
                        _dp(sg) if sg is not None else None, q, _dp(xr),
                        trait.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(b),
                        int(nthreads), ctypes.byref(bad))
    if rc == -1:
        raise ValueError("oracle_gls: bad arguments")
    if rc == -3:
        raise MemoryError("oracle_gls: allocation failed")
    if rc <= -2:
        raise OracleError("oracle_gls: M_j is not SPD for trait %d" % (-2 - rc))
    return (b, int(bad.value)) if return_non_spd else b


def gls_grid(phi, xl, xr, y, h2, sigma2=None, nthreads: int = 0):
    """Full grid: every SNP of xr [m][n] against every trait of y [t][n] -> b [m][t][p]."""
    xr = np.atleast_2d(xr)
    y = np.atleast_2d(y)
    m, t = xr.shape[0], y.shape[0]
    ii = np.repeat(np.arange(m), t)
    jj = np.tile(np.arange(t), m)
    b = gls(phi, xl, xr[ii], y, h2, trait=jj, sigma2=sigma2, nthreads=nthreads)
    return b.reshape(m, t, -1)


def relative_error(b_hat, b_ref):
    """Per-problem relative error ||b_hat - b_ref||_2 / ||b_ref||_2 over the last axis."""
    b_hat = np.asarray(b_hat, dtype=np.float64)
    b_ref = np.asarray(b_ref, dtype=np.float64)
    return np.linalg.norm(b_hat - b_ref, axis=-1) / np.linalg.norm(b_ref, axis=-1)
