"""Shared helpers of the GPU tests: build a cohort on cuda:0 from synthetic inputs."""
import numpy as np

import oracle
from paper_1210_7683_amd import gwas

# Error bounds of b against the FP64 oracle, per form: FP64 and FP32 are the
# stated targets; the three-piece split BF16 form carries the FP32 value exactly
# and drops products below FP32 rounding, so it takes the FP32 target; the
# two-piece form's bound is the measured one over every problem of the
# paper-shape grids (largest 3.9e-4 at m = 1e5, on a trait whose ||b|| is a
# twentieth of the median), with margin.
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x3": 1e-3, "bf16x6": 1e-5}


def grid_error_vs(b, b64, chunk=100_000):
    """Per-problem ||b - b64|| / ||b64|| over a whole device grid [m][t][p], in
    SNP chunks; returns (max, argmax (i, j), error tensor [m][t] float32)."""
    import torch
    m, t = b.shape[0], b.shape[1]
    e = torch.empty((m, t), dtype=torch.float32, device=b.device)
    for i0 in range(0, m, chunk):
        r = b64[i0:i0 + chunk]
        d = b[i0:i0 + chunk].double() - r
        e[i0:i0 + chunk] = (torch.linalg.vector_norm(d, dim=-1) / torch.linalg.vector_norm(r, dim=-1)).float()
    mx, am = e.reshape(-1).max(0)
    return float(mx), divmod(int(am), t), e
ALL_FORMS = ("f64", "f32", "bf16x3", "bf16x6")


def rel_err(b_hat, b_ref):
    """Per-problem relative error ||b_hat - b||_2 / ||b||_2."""
    return oracle.relative_error(b_hat, b_ref)


def scaled_err(b_hat, b_ref, trait_axis=1):
    """Per-problem error relative to max(||b||, median ||b|| over the trait's problems).

    When a trait carries no signal at a SNP, b is close to zero and its
    relative error measures the rounding floor of the sums divided by ||b||;
    flooring the denominator at the trait's typical ||b|| keeps the measure
    about the arithmetic, not about how close to zero a particular b falls.
    """
    b_hat = np.asarray(b_hat, dtype=np.float64)
    b_ref = np.asarray(b_ref, dtype=np.float64)
    nb = np.linalg.norm(b_ref, axis=-1)
    if trait_axis is None or nb.ndim < 2:   # one pooled median (a list of sampled problems)
        med = np.median(nb)
    else:
        med = np.median(nb, axis=tuple(a for a in range(nb.ndim) if a != trait_axis), keepdims=True)
    return np.linalg.norm(b_hat - b_ref, axis=-1) / np.maximum(nb, med)


def check_bound(b_hat, b_ref, form, bound=None, label=""):
    """Assert a form's bound on b against a reference (problems along the last
    axis but one, traits on axis 1 when b has three axes).

    FP64: every problem's relative error ||b_hat - b|| / ||b|| is at most the
    bound (1e-10 unless given). Reduced forms: the error scaled by
    max(||b||, the trait's median ||b||) is at most the bound everywhere, and
    the relative error at its 99th percentile; a pure-noise trait can have a
    b close to zero, whose relative error is then the rounding floor of the
    form's sums divided by ||b||. Returns (relative, scaled) errors."""
    bound = TOL[form] if bound is None else bound
    rel = rel_err(b_hat, b_ref)
    sc = scaled_err(b_hat, b_ref)
    print("%s%s: relative max %.3e median %.3e, scaled max %.3e (bound %.0e)" % (
        label + " " if label else "", form, rel.max(), np.median(rel), sc.max(), bound))
    if form == "f64":
        assert rel.max() <= bound, (label, form, rel.max())
    else:
        assert sc.max() <= bound, (label, form, sc.max())
        assert np.quantile(rel, 0.99) <= bound, (label, form, np.quantile(rel, 0.99))
    return rel, sc


def cohort(phi, xl, xr, forms=ALL_FORMS, m_capacity=None, **kw):
    w, z = np.linalg.eigh(phi)
    c = gwas.Cohort(z, w, xl, m_capacity or xr.shape[0], forms=forms, **kw)
    c.rotate(0, xr)
    return c
