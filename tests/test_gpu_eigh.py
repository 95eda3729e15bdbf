"""Setup-time eigendecomposition on the device (gwas_eigh): an
eigendecomposition of Phi to FP64 accuracy, the same from host and device
memory, and a cohort built on it solves the grid within the forms' bounds of
the oracle (which factorises every M_j from Phi itself)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import check_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _spd(n, seed):
    if n < 8:
        a = np.random.default_rng(seed).standard_normal((n, n + 3))
        return a @ a.T / (n + 3) + 1e-3 * np.eye(n)
    return synth.small(n, 2, 1, 1, seed=seed)[0]


@pytest.mark.parametrize("n", [1, 7, 128, 1000])
def test_device_eigh_is_an_eigendecomposition(n, torch_cuda):
    torch = torch_cuda
    from paper_1210_7683_amd import gwas
    phi = _spd(n, seed=n)
    w, z = gwas.eigh(phi)
    w_ref = np.linalg.eigvalsh(phi)
    scale = np.abs(w_ref).max()
    print("n=%d: eigenvalues %.2e, residual %.2e, orthogonality %.2e" % (
        n, np.abs(w - w_ref).max() / scale, np.abs(phi @ z - z * w).max() / scale,
        np.abs(z.T @ z - np.eye(n)).max()))
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - w_ref).max() <= 1e-12 * scale
    assert np.abs(phi @ z - z * w).max() <= 1e-12 * scale
    assert np.abs(z.T @ z - np.eye(n)).max() <= 1e-12
    wd, zd = gwas.eigh(torch.from_numpy(phi).cuda())
    assert wd.is_cuda and zd.is_cuda
    assert np.abs(wd.cpu().numpy() - w).max() <= 1e-14 * scale
    assert np.abs(np.abs(zd.cpu().numpy()) - np.abs(z)).max() <= 1e-10


def test_solve_from_the_device_eigendecomposition_against_oracle(torch_cuda):
    from paper_1210_7683_amd import gwas
    phi, xl, xr, y, h2 = synth.small(300, 4, 200, 8, seed=5)
    w, z = gwas.eigh(phi)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = gwas.Cohort(z, w, xl, 200, forms=("f64", "f32", "bf16x6"))
    c.rotate(0, xr)
    for form in ("f64", "f32", "bf16x6"):
        b = c.solve(y, h2, form=form).cpu().numpy()
        check_bound(b, ref, form, label="device eigendecomposition")
    c.close()


def test_eigh_argument_errors(torch_cuda):
    from paper_1210_7683_amd import gwas
    with pytest.raises(ValueError):
        gwas.eigh(np.zeros((3, 4)))
    with pytest.raises(gwas.GwasError, match="outside"):
        gwas.eigh(np.zeros((0, 0)))
