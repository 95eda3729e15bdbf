"""Test infrastructure only: Eq. (1) evaluated through the eigendecomposition of Phi.

A second FP64 reference, independent of both the C oracle and the GPU path.
It rests on one identity of Section 3.1: with Phi = Z diag(w) Z^T and
Z orthogonal, M_j = h2_j Phi + (1 - h2_j) I = Z diag(h2_j w + 1 - h2_j) Z^T,
so M_j^{-1} = Z diag(d_j) Z^T with d_j = 1 / (h2_j w + 1 - h2_j). Substituted
into Eq. (1), every product X^T M_j^{-1} X' becomes (Z^T X)^T diag(d_j) (Z^T X'):
the design matrix X_i = [X_L | x_i] and the trait y_j are rotated by Z^T once,
and each problem is a weighted least-squares problem in the rotated basis,

    G_ij = A_i^T diag(d_j) A_i,   r_ij = A_i^T diag(d_j) (Z^T y_j),   G_ij b_ij = r_ij,

with A_i = Z^T X_i (n x p). This module forms G_ij and r_ij whole for each
problem and solves them with numpy's LU solve; it takes none of the paper's
partitioning of G into covariate and SNP blocks and no square roots of d_j.
"""
from __future__ import annotations

import numpy as np


def gls_rotated(xl, xr, y, h2, z, w):
    """b [m][t][p] for X_L [(p-1)][n], X_R [m][n], Y [t][n], h2 [t] and
    Phi = Z diag(w) Z^T (Z orthogonal, eigenvectors in columns)."""
    xl = np.atleast_2d(np.asarray(xl, dtype=np.float64))
    xr = np.atleast_2d(np.asarray(xr, dtype=np.float64))
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    h2 = np.atleast_1d(np.asarray(h2, dtype=np.float64))
    z = np.asarray(z, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    m, t, n = xr.shape[0], y.shape[0], z.shape[0]
    p = xl.shape[0] + 1
    # A_i = Z^T [X_L | x_i] for every SNP, stacked: a[i] is n x p
    a = np.empty((m, n, p))
    a[:, :, : p - 1] = (z.T @ xl.T)[None, :, :]
    a[:, :, p - 1] = xr @ z
    yr = y @ z                                  # row j = (Z^T y_j)^T
    b = np.empty((m, t, p))
    for j in range(t):
        d = 1.0 / (h2[j] * w + (1.0 - h2[j]))   # M_j^{-1} = Z diag(d) Z^T
        da = a * d[None, :, None]               # diag(d) A_i
        g = np.matmul(a.transpose(0, 2, 1), da)        # G_ij, m x p x p
        r = np.matmul(da.transpose(0, 2, 1), yr[j])    # r_ij, m x p
        b[:, j, :] = np.linalg.solve(g, r[..., None])[..., 0]
    return b
