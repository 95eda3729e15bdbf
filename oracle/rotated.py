"""Test infrastructure only: the paper's eigendecomposition-based reduction on the CPU.

A second FP64 reference, independent of both the C oracle and the GPU path,
written from Section 3 of the paper (Algorithms 1, 2 and 5):

  Phi = Z Lambda Z^T;  X'_L = Z^T X_L;  X'_R = Z^T X_R;  Y' = Z^T Y;
  per trait j:  D_j = sigma2_j (h2_j Lambda + (1 - h2_j) I),  K_j = D_j^{-1/2},
                W_L = K_j X'_L,  v_j = K_j y'_j,  S_TL = W_L^T W_L,  b_T = W_L^T v_j;
  per SNP i:    W_R = K_j x'_i,  S_BL = W_R^T W_L,  S_BR = W_R^T W_R,  b_B = W_R^T v_j,
                b_ij = S_ij^{-1} [b_T; b_B],  S_ij = [[S_TL, S_BL^T], [S_BL, S_BR]].

The paper writes K_j K_j^T = D_j^{-1/2} in its listings but defines
K_j := D_j^{-1/2} in the text; the text's reading (K_j K_j^T = D_j^{-1}) is the
one that reproduces Eq. (1), and is used here.
"""
from __future__ import annotations

import numpy as np


def eig(phi):
    """Phi = Z diag(lam) Z^T (Algorithm 5, first preloop step)."""
    lam, z = np.linalg.eigh(np.asarray(phi, dtype=np.float64))
    return z, lam


def mt_gwas(xl, xr, y, h2, z, lam, sigma2=None):
    """b [m][t][p] for X_L [(p-1)][n], X_R [m][n], Y [t][n], h2 [t], Phi = Z diag(lam) Z^T."""
    xl = np.atleast_2d(np.asarray(xl, dtype=np.float64))
    xr = np.atleast_2d(np.asarray(xr, dtype=np.float64))
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    h2 = np.atleast_1d(np.asarray(h2, dtype=np.float64))
    sigma2 = np.ones_like(h2) if sigma2 is None else np.atleast_1d(np.asarray(sigma2, dtype=np.float64))
    m, t, p = xr.shape[0], y.shape[0], xl.shape[0] + 1
    xlp = z.T @ xl.T            # X'_L  n x (p-1)
    xrp = z.T @ xr.T            # X'_R  n x m
    yp = z.T @ y.T              # Y'    n x t
    b = np.empty((m, t, p))
    for j in range(t):
        d = sigma2[j] * (h2[j] * lam + (1.0 - h2[j]))      # D_j
        k = 1.0 / np.sqrt(d)                                # K_j = D_j^{-1/2}
        wl = k[:, None] * xlp                               # W_L   n x (p-1)
        v = k * yp[:, j]                                    # v_j
        stl = wl.T @ wl                                     # S_TL
        bt = wl.T @ v                                       # b_T
        wr = k[:, None] * xrp                               # W_R for every SNP, n x m
        sbl = wr.T @ wl                                     # S_BL  m x (p-1)
        sbr = np.einsum("ki,ki->i", wr, wr)                 # S_BR  m
        bb = wr.T @ v                                       # b_B   m
        s = np.empty((m, p, p))
        s[:, : p - 1, : p - 1] = stl
        s[:, p - 1, : p - 1] = sbl
        s[:, : p - 1, p - 1] = sbl
        s[:, p - 1, p - 1] = sbr
        rhs = np.empty((m, p))
        rhs[:, : p - 1] = bt
        rhs[:, p - 1] = bb
        b[:, j, :] = np.linalg.solve(s, rhs[..., None])[..., 0]
    return b
