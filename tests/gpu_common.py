"""Shared helpers of the GPU tests: build a cohort on cuda:0 from synthetic inputs."""
import numpy as np

import oracle
from paper_1210_7683_amd import gwas

# Per-problem relative 2-norm error bounds of b against the FP64 oracle.
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x3": 2e-3}


def rel_err(b_hat, b_ref):
    return oracle.relative_error(b_hat, b_ref)


def cohort(phi, xl, xr, forms=("f64", "f32", "bf16x3"), m_capacity=None, **kw):
    w, z = np.linalg.eigh(phi)
    c = gwas.Cohort(z, w, xl, m_capacity or xr.shape[0], forms=forms, **kw)
    c.rotate(0, xr)
    return c
