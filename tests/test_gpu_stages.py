"""Stage-by-stage checks of the HIP path against numpy FP64 (rotation, trait prologue, panels).

These isolate each kernel's error before the end-to-end parity tests: the
rotated covariates X'_L = Z^T X_L, the rotated traits, the per-trait factors
L_j^{-1} and z_j = L_j^{-1} b_T_j of S_TL_j = X'_L^T diag(d_j) X'_L
(Algorithm 5, trait loop), and the contraction panels d_j, d_j o x'_L, d_j o y'_j.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import cohort

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup_small():
    import torch
    assert torch.cuda.is_available()
    n, p, m, t = 100, 4, 40, 6
    phi, xl, xr, y, h2 = synth.small(n, p, m, t, seed=21)
    w, z = np.linalg.eigh(phi)
    c = cohort(phi, xl, xr, max_traits=8)
    c.solve(y, h2, form="f64")
    yield dict(n=n, p=p, t=t, xl=xl, y=y, h2=h2, w=w, z=z, c=c)
    c.close()


def test_rotated_covariates(setup_small):
    d = setup_small
    npad = 128
    got = d["c"].debug_copy("xl").reshape(d["p"] - 1, npad)
    ref = d["xl"] @ d["z"]
    assert np.allclose(got[:, : d["n"]], ref, rtol=0, atol=1e-12)
    assert not got[:, d["n"]:].any()


def test_rotated_traits(setup_small):
    d = setup_small
    got = d["c"].debug_copy("yt").reshape(8, 128)[: d["t"]]
    ref = d["y"] @ d["z"]
    assert np.allclose(got[:, : d["n"]], ref, rtol=0, atol=1e-12)


def test_trait_factors(setup_small):
    d = setup_small
    q = d["p"] - 1
    ntl = q * (q + 1) // 2
    stride = (ntl + q + 1) & ~1
    got = d["c"].debug_copy("fac").reshape(8, stride)[: d["t"]]
    xlp = d["xl"] @ d["z"]            # [q][n]
    yp = d["y"] @ d["z"]
    for j in range(d["t"]):
        dj = 1.0 / (d["h2"][j] * d["w"] + 1 - d["h2"][j])
        stl = (xlp * dj) @ xlp.T
        bt = (xlp * dj) @ yp[j]
        linv = np.linalg.inv(np.linalg.cholesky(stl))
        z = linv @ bt
        packed = np.array([linv[a, b] for a in range(q) for b in range(a + 1)])
        assert np.allclose(got[j, :ntl], packed, rtol=1e-12, atol=1e-14), j
        assert np.allclose(got[j, ntl : ntl + q], z, rtol=1e-11, atol=1e-13), j


def test_f64_panels(setup_small):
    d = setup_small
    p, n = d["p"], d["n"]
    got = d["c"].debug_copy("panels", "f64").reshape(p + 1, 16, 128)   # planes of 8 traits padded to 16 rows
    xlp = d["xl"] @ d["z"]
    yp = d["y"] @ d["z"]
    for j in range(d["t"]):
        dj = 1.0 / (d["h2"][j] * d["w"] + 1 - d["h2"][j])
        assert np.allclose(got[0, j, :n], dj, rtol=1e-15)
        for c in range(p - 1):
            assert np.allclose(got[1 + c, j, :n], dj * xlp[c], rtol=1e-12, atol=1e-13)
        assert np.allclose(got[p, j, :n], dj * yp[j], rtol=1e-12, atol=1e-13)
    assert not got[:, :d["t"], n:].any()


def _unfragment(plane, rows, n_pad):
    """A split-BF16 plane in MFMA fragment order -> [rows][n_pad]: the 1 KB block
    (row // 16, k // 32) holds lane L = ((k % 32) // 8) * 16 + row % 16 at
    elements 8 L .. 8 L + 7 (samples 8 ((k % 32) // 8) .. + 7 of that row)."""
    b = plane.reshape(rows // 16, n_pad // 32, 4, 16, 8)      # [row group][k group][k quarter][row][k]
    return b.transpose(0, 3, 1, 2, 4).reshape(rows, n_pad)


def test_split_bf16_panels_in_fragment_order(setup_small):
    """The two-piece form's panels (hi and lo planes per contraction) in fragment
    order: hi + lo is the FP32 rounding of the FP64 panel value to within BF16's
    two-piece precision, and samples beyond n are zero."""
    d = setup_small
    p, n = d["p"], d["n"]
    d["c"].solve(d["y"], d["h2"], form="bf16x3")
    raw = d["c"].debug_copy("panels", "bf16x3").reshape(2 * (p + 1), 16 * 128)
    val = lambda u: (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    planes = np.stack([_unfragment(raw[k], 16, 128) for k in range(2 * (p + 1))])
    xlp = d["xl"] @ d["z"]
    yp = d["y"] @ d["z"]
    for j in range(d["t"]):
        dj = 1.0 / (d["h2"][j] * d["w"] + 1 - d["h2"][j])
        refs = [dj] + [dj * xlp[c] for c in range(p - 1)] + [dj * yp[j]]
        for q, ref in enumerate(refs):
            got = val(planes[2 * q, j, :n]) + val(planes[2 * q + 1, j, :n])
            assert np.abs(got - ref).max() <= 2.0 ** -16 * np.abs(ref).max(), (j, q)
            assert not planes[2 * q : 2 * q + 2, j, n:].any()
    d["c"].solve(d["y"], d["h2"], form="f64")   # leave the f64 panels for other tests
