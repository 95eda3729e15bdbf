"""gwas_solve_noalloc (the entry point that allocates nothing) against gwas_solve.

Both run the same kernels, so b must agree bitwise; two calls in a row, the
second smaller (fewer SNPs from an offset, fewer traits given as a device
tensor: the dot-product kernel in the FP64 and FP32 forms), so stale contents
of the shared array would show. A large-n cohort makes the array hold fewer
traits than the call has (two trait sub-blocks inside the call).
"""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_common import ALL_FORMS, cohort

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form", ALL_FORMS)
def test_noalloc_equals_solve_on_two_calls(form):
    import torch
    assert torch.cuda.is_available()
    phi, xl, xr, y, h2 = synth.small(200, 4, 700, 50, seed=2024)
    c = cohort(phi, xl, xr, forms=(form,))
    dt = torch.float64 if form == "f64" else torch.float32
    for i0, m, t, ydev in [(0, 700, 50, False), (37, 300, 2, True)]:
        yy = torch.from_numpy(y[:t]).cuda() if ydev else y[:t]
        ref = c.solve(yy, h2[:t], form=form, i0=i0, m=m)
        out = torch.full((m, t, 4), float("nan"), dtype=dt, device="cuda")
        c.solve_noalloc(yy, h2[:t], out, form=form, i0=i0)
        torch.cuda.synchronize()
        print("%s i0=%d m=%d t=%d: max |noalloc - solve| = %.3g" % (
            form, i0, m, t, float((out.double() - ref.double()).abs().max())))
        assert bool(torch.isfinite(out).all())
        assert torch.equal(out, ref)
    c.close()


def test_noalloc_trait_sub_blocks_and_errors():
    """n = 4096, FP64: about 146 traits fit the array per sub-block, so 200
    traits take two; b equals gwas_solve's (one sub-block). A host b is refused."""
    import torch
    from paper_1210_7683_amd import gwas
    phi, xl, xr, y, h2 = synth.small(4096, 4, 300, 200, seed=4097, k=4096)
    c = cohort(phi, xl, xr, forms=("f64",))
    ref = c.solve(y, h2, form="f64")
    out = torch.full_like(ref, float("nan"))
    c.solve_noalloc(y, h2, out, form="f64")
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    host = np.empty((300, 200, 4))
    st = gwas.load().gwas_solve_noalloc(c._h, 0, 300, 200, y.ctypes.data, 0, np.ascontiguousarray(h2).ctypes.data,
                                        gwas.FORM_F64, ctypes.c_void_p(host.ctypes.data), None)
    assert st == gwas.EINVAL
    assert "device memory" in gwas.load().gwas_last_error().decode()
    c.close()
