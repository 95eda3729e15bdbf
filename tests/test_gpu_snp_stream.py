"""Genotype stream (gwas_solve_snp_stream): SNPs that are not resident pass
through the rotated store block by block; b must equal, bitwise, that of
rotating every SNP into a resident store and solving there, and match the
oracle at the form's tolerance."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import ALL_FORMS, check_bound, cohort

pytestmark = pytest.mark.gpu

FORMS = list(ALL_FORMS)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def collect(c, xr, y, h2, form, **kw):
    m, t = xr.shape[0], y.shape[0]
    dt = np.float64 if form == "f64" else np.float32
    b = np.full((m, t, c.p), np.nan, dtype=dt)
    seen = np.zeros((m, t), dtype=np.int32)

    def on_slab(info, arr):
        i0, cnt, j0, tb = info["i0"], info["count"], info["j0"], info["tb"]
        b[i0:i0 + cnt, j0:j0 + tb] = arr
        seen[i0:i0 + cnt, j0:j0 + tb] += 1
        from paper_1210_7683_amd import gwas
        assert gwas.checksum(arr) == info["checksum"]

    sums = c.solve_snp_stream(xr, y, h2, form=form, on_slab=on_slab, **kw)
    assert (seen == 1).all()   # every problem delivered exactly once
    return b, sums


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,p,m,t,cap,slab,traits,chunk", [(200, 4, 1000, 7, 256, 64, 1024, 0),
                                                            (77, 3, 301, 40, 64, 16, 16, 0),
                                                            (130, 5, 250, 2, 100, 32, 1024, 0),
                                                            (200, 4, 1500, 7, 1024, 64, 1024, 256)])
def test_streamed_snps_equal_resident_solve(form, n, p, m, t, cap, slab, traits, chunk, torch_cuda):
    """chunk > 0: the genotype blocks (cap / 2 SNPs) are repacked and rotated
    chunk SNPs at a time on the library's second stream (geno_chunk_snps)."""
    torch = torch_cuda
    phi, xl, xr, y, h2 = synth.small(n, p, m, t, seed=n + m + t)
    ref_c = cohort(phi, xl, xr, forms=(form,), max_traits=traits)
    full = ref_c.solve(y, h2, form=form).cpu().numpy()
    ref_c.close()
    w, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    c = gwas.Cohort(z, w, xl, cap, forms=(form,), slab_snps=slab, max_traits=traits, geno_chunk_snps=chunk)
    host = torch.from_numpy(xr).pin_memory()
    b, sums = collect(c, host, y, h2, form)
    assert np.array_equal(b, full)
    st = c.stats()
    assert st["snps_rotated"] == m and st["problems"] == m * t
    # the same call from a device copy of the genotypes
    b2, sums2 = collect(c, torch.from_numpy(xr).cuda(), y, h2, form)
    assert np.array_equal(b2, full) and sums2 == sums
    c.close()
    check_bound(b, oracle.gls_grid(phi, xl, xr, y, h2), form, label="SNP stream n=%d p=%d" % (n, p))


def test_snp_stream_argument_errors(torch_cuda):
    phi, xl, xr, y, h2 = synth.small(64, 2, 10, 2, seed=3)
    w, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    c1 = gwas.Cohort(z, w, xl, 1, forms=("f32",))
    with pytest.raises(gwas.GwasError, match="at least 2"):
        c1.solve_snp_stream(xr, y, h2, form="f32")
    c1.close()
    c = gwas.Cohort(z, w, xl, 4, forms=("f32",))
    assert c.solve_snp_stream(xr[:0], y, h2, form="f32") == []
    with pytest.raises(gwas.GwasError, match="not resident"):
        c.solve_snp_stream(xr, y, h2, form="f64")
    with pytest.raises(ValueError):
        c.solve_snp_stream(xr[:, :10], y, h2, form="f32")
    c.close()
