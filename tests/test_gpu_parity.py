"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every test here runs the kernels on cuda:0 and compares b element by element
with the oracle (oracle/oracle.c, a dense-Cholesky solve of Eq. (1)) on the
same seeded inputs, to the per-form bound: FP64 1e-10, FP32 and three-piece
split BF16 1e-5, two-piece split BF16 1e-3 (its measured bound over whole
paper-shape grids, with margin). The FP64 form's bound applies to every
problem's relative error ||b_hat - b|| / ||b|| in every test, and so do the
reduced forms' bounds on the paper-shaped workloads (p = 4). On the ragged
shapes (p from 2 to 20, short n) the reduced forms are bounded in the error
scaled by max(||b||, the trait's median ||b||) and in the 99th percentile of
the relative error, since with p = 2 a few problems out of thousands have
||b|| near zero and their relative error is the rounding floor of the form's
sums divided by ||b|| (reported, not bounded).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import ALL_FORMS, TOL, check_bound, cohort, grid_error_vs, rel_err, scaled_err

pytestmark = pytest.mark.gpu

FORMS = list(ALL_FORMS)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def tiny(torch_cuda):
    w = synth.WORKLOADS["tiny"]
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = cohort(phi, xl, xr)
    yield dict(phi=phi, xl=xl, xr=xr, y=y, h2=h2, ref=ref, c=c)
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_tiny_full_grid(tiny, form, torch_cuda):
    b = tiny["c"].solve(tiny["y"], tiny["h2"], form=form).cpu().numpy()
    err = rel_err(b, tiny["ref"])
    print("tiny %s: max %.3e median %.3e" % (form, err.max(), np.median(err)))
    assert b.shape == (512, 8, 4)
    assert np.isfinite(b).all()
    assert err.max() <= TOL[form]


def test_rotation_matches_fp64_gemm(tiny, torch_cuda):
    w, z = np.linalg.eigh(tiny["phi"])
    xr = tiny["xr"]
    ref = xr.astype(np.float64) @ z          # row i = (Z^T x_i)^T
    got = tiny["c"].copy_rotated(0, xr.shape[0], "f64")
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    got32 = tiny["c"].copy_rotated(0, xr.shape[0], "f32")
    assert np.array_equal(got32, got.astype(np.float32))


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.uint8])
def test_rotate_dtypes_and_device_input(tiny, dtype, torch_cuda):
    torch = torch_cuda
    xr = tiny["xr"][:100].astype(dtype)
    w, z = np.linalg.eigh(tiny["phi"])
    from paper_1210_7683_amd import gwas
    c = gwas.Cohort(z, w, tiny["xl"], 300, forms=("f64",))
    c.rotate(7, xr)                                   # host block
    c.rotate(150, torch.from_numpy(xr).cuda())        # device block
    torch.cuda.synchronize()
    a = c.copy_rotated(7, 100, "f64")
    b = c.copy_rotated(150, 100, "f64")
    assert np.array_equal(a, b)
    ref = xr.astype(np.float64) @ z
    assert np.abs(a - ref).max() <= 1e-12 * np.abs(ref).max()
    c.close()


@pytest.mark.parametrize("full", [True, False])
@pytest.mark.parametrize("n,m,shift,chunk", [(1000, 300, 0, 0), (333, 257, 0, 0), (1000, 300, 1, 0), (64, 17, 0, 0),
                                             (600, 1100, 0, 0), (600, 1100, 1, 0), (1000, 700, 0, 256),
                                             (333, 1100, 1, 512)])
def test_genotype_rotation_full_byte_range(n, m, shift, chunk, full, torch_cuda):
    """Genotype bytes over the whole range 0..255 (the int8 kernels offset them
    to v - 128 and sum exact int32 digit products): every rotated value against
    the FP64 product. The rows are repacked on the device before the int8
    kernel: a word at a time where n, the stride and the address are multiples
    of 4 (n = 1000, 600, 64), byte by byte for n = 333 and for rows starting at
    an odd device address (shift = 1). chunk > 0 repacks that many rows at a
    time (geno_chunk_snps), so several chunks and a ragged last one are taken.
    n = 600, m = 1100: 10 or 20 column tiles and 9 row tiles, so the tile order's
    tail (column tiles past the last multiple of 8, by groups of 8 row tiles)
    and its partial group are taken.
    With an FP64 store (full) all six Z digits are used and the FP64 values are
    checked to 1e-12 of the maximum; without one, the leading four, and the
    FP32 values are checked to 1e-7 of the maximum (FP32 rounding is 6e-8)."""
    torch = torch_cuda
    phi, xl, _, _, _ = synth.small(n, 3, 1, 1, seed=n + shift)
    xr = np.random.default_rng(n + m).integers(0, 256, size=(m, n), dtype=np.uint8)
    xr[0] = 255                       # extreme rows
    xr[1] = 0
    w, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    c = gwas.Cohort(z, w, xl, m, forms=("f64", "f32") if full else ("f32",), geno_chunk_snps=chunk)
    buf = torch.zeros(m * n + shift, dtype=torch.uint8, device="cuda")
    dev = buf[shift:].view(m, n)
    dev.copy_(torch.from_numpy(xr))
    assert dev.data_ptr() % 4 == shift
    c.rotate(0, dev)
    torch.cuda.synchronize()
    ref = xr.astype(np.float64) @ z
    if full:
        got = c.copy_rotated(0, m, "f64")
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert np.array_equal(c.copy_rotated(0, m, "f32"), got.astype(np.float32))
    else:
        err = np.abs(c.copy_rotated(0, m, "f32").astype(np.float64) - ref).max() / np.abs(ref).max()
    print("n=%d m=%d shift=%d chunk=%d full=%d: max |rotated - FP64 product| / max = %.2e" % (
        n, m, shift, chunk, full, err))
    assert err <= (1e-12 if full else 1e-7)
    c.close()


def test_genotype_rotation_in_pieces_at_offsets(torch_cuda):
    """Genotype blocks rotated into the middle of the store, in repack chunks of
    256 SNPs (chunk offsets add to the block's first row), give the same store,
    bitwise, as one call over all SNPs; both against the FP64 product."""
    torch = torch_cuda
    n, m = 333, 1100
    phi, xl, _, _, _ = synth.small(n, 3, 1, 1, seed=8)
    xr = np.random.default_rng(9).integers(0, 256, size=(m, n), dtype=np.uint8)
    w, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    whole = gwas.Cohort(z, w, xl, m, forms=("f64",), geno_chunk_snps=256)
    whole.rotate(0, torch.from_numpy(xr).cuda())
    pieces = gwas.Cohort(z, w, xl, m, forms=("f64",), geno_chunk_snps=256)
    for a, b in [(700, 1100), (0, 300), (300, 700)]:   # out of order, each spanning chunks
        pieces.rotate(a, torch.from_numpy(np.ascontiguousarray(xr[a:b])).cuda())
    torch.cuda.synchronize()
    got_whole, got_pieces = whole.copy_rotated(0, m, "f64"), pieces.copy_rotated(0, m, "f64")
    whole.close()
    pieces.close()
    assert np.array_equal(got_whole, got_pieces)
    ref = xr.astype(np.float64) @ z
    assert np.abs(got_pieces - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_full_byte_range_genotypes_solve_against_oracle(form, torch_cuda):
    """b for genotype bytes over 0..255 (dosages scaled to a byte, say) against
    the oracle, at the form's bound."""
    phi, xl, _, y, h2 = synth.small(200, 4, 1, 6, seed=17)
    xr = np.random.default_rng(18).integers(0, 256, size=(150, 200), dtype=np.uint8)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = cohort(phi, xl, xr, forms=(form,))
    b = c.solve(y, h2, form=form).cpu().numpy()
    c.close()
    check_bound(b, ref, form, label="bytes 0..255")


@pytest.mark.parametrize("n,m", [(77, 129), (200, 333), (1000, 300)])
def test_genotype_rotation_ragged_n_and_rows(n, m, torch_cuda):
    """uint8 genotypes with n not a multiple of the 64-sample stage (and, for
    n = 77, rows not 8-byte aligned), rows not a multiple of the SNP tile:
    every rotated value against the FP64 product, in all three stores."""
    torch = torch_cuda
    phi, xl, xr, _, _ = synth.small(n, 3, m, 2, seed=n + m)
    assert xr.dtype == np.uint8
    w, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    c = gwas.Cohort(z, w, xl, m + 5)
    c.rotate(5, torch.from_numpy(xr).cuda())
    torch.cuda.synchronize()
    ref = xr.astype(np.float64) @ z
    got = c.copy_rotated(5, m, "f64")
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(c.copy_rotated(5, m, "f32"), got.astype(np.float32))
    c.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,p,m,t", [(200, 2, 333, 37), (77, 3, 100, 5), (130, 5, 129, 17),
                                     (96, 8, 70, 33), (64, 13, 40, 9), (150, 20, 35, 18),
                                     (128, 4, 1100, 150)])
def test_ragged_shapes_and_p(form, n, p, m, t, torch_cuda):
    phi, xl, xr, y, h2 = synth.small(n, p, m, t, seed=n * 31 + p)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = cohort(phi, xl, xr, forms=(form,))
    b = c.solve(y, h2, form=form).cpu().numpy()
    c.close()
    check_bound(b, ref, form, label="n=%d p=%d m=%d t=%d" % (n, p, m, t))


def test_fp32_without_fp64_folds(torch_cuda):
    """f32_flush = 0: the FP32 form accumulates the whole K loop in FP32 (no FP64
    folds). No bound is stated for this variant; it is checked against ten times
    the FP32 bound, against the default (folded) result, which must differ from it
    and be at least as accurate over the grid, at a ragged n over several stages
    and trait tiles."""
    phi, xl, xr, y, h2 = synth.small(333, 4, 300, 40, seed=3301)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c0 = cohort(phi, xl, xr, forms=("f32",), f32_flush=0)
    b0 = c0.solve(y, h2, form="f32").cpu().numpy()
    c0.close()
    c2 = cohort(phi, xl, xr, forms=("f32",))
    b2 = c2.solve(y, h2, form="f32").cpu().numpy()
    c2.close()
    e0, e2 = scaled_err(b0, ref), scaled_err(b2, ref)
    print("n=333 f32 without folds: scaled max %.3e median %.3e; with folds: max %.3e median %.3e" % (
        e0.max(), np.median(e0), e2.max(), np.median(e2)))
    assert e0.max() <= 10 * TOL["f32"]
    assert e2.max() <= TOL["f32"]
    assert not np.array_equal(b0, b2)
    assert np.median(e2) <= np.median(e0)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,p,m,t", [(200, 2, 333, 1), (77, 4, 100, 2), (130, 9, 129, 3),
                                     (1000, 4, 70, 1), (1000, 4, 70, 2), (1000, 4, 1100, 3),
                                     (1000, 9, 70, 3), (1000, 4, 70, 4), (64, 20, 40, 1),
                                     (96, 13, 65, 3)])
def test_small_trait_calls_use_the_dot_product_kernel(form, n, p, m, t, torch_cuda):
    """FP64 and FP32 solve calls with t <= 3 traits whose panels fit the 160 KB
    of LDS run the dot-product kernel (counted in the stats): with 256-thread
    workgroups while the panels take at most 40 KB, else 1024 (n = 1000, p = 4:
    FP64 t = 2, 3 and FP32 t = 3); FP64 at p = 9, t = 3 (240 KB) keeps the MFMA
    tiles. Every case: parity with the oracle at the form's tolerance, ragged m
    and n, and the device, sub-range and host-slab outputs agree bitwise."""
    torch = torch_cuda
    phi, xl, xr, y, h2 = synth.small(n, p, m, t, seed=n * 7 + p + t)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = cohort(phi, xl, xr, forms=(form,), slab_snps=32)
    b = c.solve(y, h2, form=form).cpu().numpy()
    n_pad = (n + 63) // 64 * 64
    dot = form in ("f64", "f32") and t <= 3 and (p + 1) * t * n_pad * (8 if form == "f64" else 4) <= 160 * 1024
    assert c.stats()["dot_launches"] == (1 if dot else 0)
    check_bound(b, ref, form, label="n=%d p=%d m=%d t=%d" % (n, p, m, t))
    part = c.solve(y, h2, form=form, i0=3, m=m - 5).cpu().numpy()
    assert np.array_equal(part, b[3:m - 2])
    dt = torch.float64 if form == "f64" else torch.float32
    host = torch.empty((m, t, p), dtype=dt, pin_memory=True)
    c.solve(y, h2, form=form, out=host)
    torch.cuda.synchronize()
    assert np.array_equal(host.numpy(), b)
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_calls_with_four_traits_use_the_mfma_tiles(form, torch_cuda):
    phi, xl, xr, y, h2 = synth.small(128, 4, 100, 4, seed=11)
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = cohort(phi, xl, xr, forms=(form,), max_traits=3)   # sub-blocks of 3 and 1 traits
    b = c.solve(y, h2, form=form).cpu().numpy()
    assert c.stats()["dot_launches"] == 0
    check_bound(b, ref, form, label="t=4 in sub-blocks of 3")
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_subranges_and_trait_subblocks_are_bitwise_consistent(form, torch_cuda):
    torch = torch_cuda
    phi, xl, xr, y, h2 = synth.small(160, 4, 300, 70, seed=5)
    c = cohort(phi, xl, xr, forms=(form,), max_traits=32)
    full = c.solve(y, h2, form=form).cpu().numpy()          # three trait sub-blocks
    part = c.solve(y, h2, form=form, i0=37, m=150).cpu().numpy()
    assert np.array_equal(part, full[37:187])
    ysub = c.solve(y[5:20], h2[5:20], form=form).cpu().numpy()
    assert np.array_equal(ysub, full[:, 5:20])
    ydev = c.solve(torch.from_numpy(y).cuda(), h2, form=form).cpu().numpy()
    assert np.array_equal(ydev, full)
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_host_output_streamed_in_slabs_equals_device_output(form, torch_cuda):
    torch = torch_cuda
    phi, xl, xr, y, h2 = synth.small(128, 4, 1000, 40, seed=9)
    c = cohort(phi, xl, xr, forms=(form,), slab_snps=96, max_traits=16)
    dev = c.solve(y, h2, form=form).cpu().numpy()
    dt = torch.float64 if form == "f64" else torch.float32
    host = torch.empty((1000, 40, 4), dtype=dt, pin_memory=True)
    c.solve(y, h2, form=form, out=host)
    torch.cuda.synchronize()
    assert np.array_equal(host.numpy(), dev)
    st = c.stats()
    assert st["bytes_d2h"] == host.numel() * host.element_size()
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_rank_deficient_snps_give_nan_and_are_counted(form, torch_cuda):
    phi, xl, xr, y, h2 = synth.small(128, 4, 20, 6, seed=2)
    cols = xr.astype(np.float64)
    cols[3] = 2.0                      # monomorphic: a multiple of the intercept
    cols[11] = xl[1]                   # a copy of a covariate
    c = cohort(phi, xl, cols, forms=(form,))
    b = c.solve(y, h2, form=form).cpu().numpy()
    assert np.isnan(b[[3, 11]]).all()
    ok = np.setdiff1d(np.arange(20), [3, 11])
    assert np.isfinite(b[ok]).all()
    assert c.stats()["non_spd"] == 2 * 6
    ref = oracle.gls_grid(phi, xl, cols[ok], y, h2)
    check_bound(b[ok], ref, form, label="full-rank SNPs beside rank-deficient ones")
    c.close()


def _schur_pivot_ratio(phi, xl, x, h2):
    """s / S_BR of the SNP column x for each trait: the share of x's weighted
    norm left once the covariates are projected out (FP64, from M_j^-1 = Z diag(d) Z^T)."""
    w, z = np.linalg.eigh(phi)
    a = z.T @ np.column_stack([xl.T, x])
    out = []
    for h in h2:
        d = 1.0 / (h * w + 1.0 - h)
        g = a.T @ (d[:, None] * a)
        q = g.shape[0] - 1
        u = np.linalg.solve(np.linalg.cholesky(g[:q, :q]), g[:q, q])
        out.append((g[q, q] - u @ u) / g[q, q])
    return np.array(out)


@pytest.mark.parametrize("form", FORMS)
def test_snps_between_the_rank_floors(form, torch_cuda):
    """SNP columns close to the span of the covariates, x = X_L c + eps r, whose
    Schur pivot ratio s / S_BR (about eps^2 |r|^2 / |x|^2) falls between the FP64
    floor (1e-10) and the reduced forms' floors (1e-4 FP32 and three-piece split
    BF16, 1e-3 two-piece). The FP64 form solves them and matches the oracle; the
    reduced forms report NaN and count them, as their sums cannot resolve the
    pivot. At ratio rho the pivot keeps about log10(1/rho) fewer digits, so two
    correct FP64 evaluations differ by about 1e-15 / rho (measured between the
    oracle and the CPU rotated reference: 3.6e-11 at rho = 3.5e-5, 2.6e-10 at
    3.1e-6): the FP64 bound is 1e-10 at rho ~ 3e-5 and 1e-8 at rho ~ 3e-6."""
    n, p, t = 128, 4, 6
    phi, xl, xr, y, h2 = synth.small(n, p, 8, t, seed=77)
    rng = np.random.default_rng(5)
    base = rng.standard_normal(p - 1) @ xl
    r = rng.standard_normal(n)
    cols = xr.astype(np.float64)
    band = {2: (1e-2, 1e-10), 5: (3e-3, 1e-8)}       # column -> (eps, FP64 bound)
    for i, (eps, _) in band.items():
        cols[i] = base + eps * r
    ratio = {i: _schur_pivot_ratio(phi, xl, cols[i], h2) for i in band}
    assert 2e-5 < ratio[2].min() and ratio[2].max() < 5e-5
    assert 2e-6 < ratio[5].min() and ratio[5].max() < 5e-6
    ref = oracle.gls_grid(phi, xl, cols, y, h2)
    assert np.isfinite(ref).all()
    c = cohort(phi, xl, cols, forms=(form,))
    b = c.solve(y, h2, form=form).cpu().numpy()
    non_spd = c.stats()["non_spd"]
    c.close()
    ok = np.setdiff1d(np.arange(8), list(band))
    check_bound(b[ok], ref[ok], form, label="full-rank SNPs beside near-dependent ones")
    if form == "f64":
        assert non_spd == 0
        for i, (eps, bound) in band.items():
            e = rel_err(b[i], ref[i])
            print("f64 pivot ratio %.1e: relative max %.3e (bound %.0e)" % (ratio[i].max(), e.max(), bound))
            assert e.max() <= bound
    else:
        assert np.isnan(b[list(band)]).all()
        assert non_spd == len(band) * t


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,p", [(3, 2), (6, 4), (17, 5)])
def test_very_few_samples(form, n, p, torch_cuda):
    """n barely above p: the whole K loop is one stage, mostly zero padding
    (n_pad = 64), against the oracle; t = 2 (the dot-product kernel in the FP64
    and FP32 forms) and t = 7 (the MFMA tiles). With n - p <= 2 the problems are
    nearly square and badly conditioned (cond(S_ij) up to 1e3 at n = 6, p = 4):
    rounding the operands to FP32 alone, with exact sums, already gives 5.4e-6
    there, so the reduced forms are held to ten times their bound; the FP64
    form and n - p >= 3 keep the bounds of the paper-shaped workloads."""
    bound = TOL[form] * (10 if n - p <= 2 and form != "f64" else 1)
    for t in (2, 7):
        phi, xl, xr, y, h2 = synth.small(n, p, 40, t, seed=n * 11 + p + t)
        ref = oracle.gls_grid(phi, xl, xr, y, h2)
        c = cohort(phi, xl, xr, forms=(form,))
        b = c.solve(y, h2, form=form).cpu().numpy()
        c.close()
        assert np.isfinite(b).all()
        check_bound(b, ref, form, bound=bound, label="n=%d p=%d t=%d" % (n, p, t))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("t", [1, 6])
def test_dependent_covariates_give_nan_for_every_problem(form, t, torch_cuda):
    """Covariates that are linearly dependent make S_TL_j singular for every
    trait (X_i never has full rank): every b is NaN and counted, as in the
    oracle; t = 1 takes the dot-product kernel in the FP64 and FP32 forms."""
    phi, xl, xr, y, h2 = synth.small(96, 4, 37, t, seed=17)
    xl = xl.copy()
    xl[2] = 3.0 * xl[1]
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    assert np.isnan(ref).all()
    c = cohort(phi, xl, xr, forms=(form,))
    b = c.solve(y, h2, form=form).cpu().numpy()
    assert np.isnan(b).all()
    assert c.stats()["non_spd"] == 37 * t
    c.close()


def test_errors_are_reported(torch_cuda):
    from paper_1210_7683_amd import gwas
    phi, xl, xr, y, h2 = synth.small(64, 4, 10, 3, seed=1)
    w, z = np.linalg.eigh(phi)
    with pytest.raises(gwas.GwasError) as e:
        gwas.Cohort(z, w, np.vstack([xl] * 7), 10)          # p = 22
    assert e.value.status == gwas.EINVAL
    c = gwas.Cohort(z, w, xl, 10, forms=("f32",))
    c.rotate(0, xr)
    for bad in [np.full(3, 1.5), np.array([0.2, -0.1, 0.3]), np.array([0.2, np.nan, 0.3])]:
        with pytest.raises(gwas.GwasError) as e:
            c.solve(y, bad, form="f32")
        assert e.value.status == gwas.EINVAL
    with pytest.raises(gwas.GwasError):
        c.solve(y, h2, form="f64")                          # form not resident
    with pytest.raises(gwas.GwasError):
        c.solve(y, h2, form="f32", i0=5, m=6)               # beyond capacity
    with pytest.raises(gwas.GwasError):
        c.rotate(8, xr[:5])
    assert c.solve(y, h2, form="f32", m=0).shape == (0, 3, 4)
    c.rotate(3, xr[:0])                                     # an empty SNP block is a no-op
    with pytest.raises(gwas.GwasError) as e:
        c.solve(y[:0], h2[:0], form="f32")                  # tb = 0
    assert e.value.status == gwas.EINVAL
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_degenerate_heritabilities_against_oracle(form, torch_cuda):
    """h2 = 0 (M = I: ordinary least squares, also checked against numpy's
    lstsq), h2 at the edges of [0, 1] and h2 = 1 (M = Phi, allowed as Phi is
    SPD), against the oracle at the form's bound."""
    phi, xl, xr, y, _ = synth.small(150, 4, 90, 6, seed=23)
    h2 = np.array([0.0, 1e-9, 0.5, 1 - 1e-9, 1.0, 0.999])
    ref = oracle.gls_grid(phi, xl, xr, y, h2)
    c = cohort(phi, xl, xr, forms=(form,))
    b = c.solve(y, h2, form=form).cpu().numpy()
    c.close()
    rel, sc = check_bound(b, ref, form, label="h2 at 0, 1 and their edges")
    print("%s: relative max per h2 %s" % (form, np.array2string(rel.max(axis=0), precision=2)))
    if form == "f64":
        for i in range(0, 90, 17):
            x = np.column_stack([xl.T, xr[i].astype(np.float64)])
            ols = np.linalg.lstsq(x, y[0], rcond=None)[0]
            assert np.abs(b[i, 0] - ols).max() <= 1e-10 * np.abs(ols).max()


@pytest.mark.parametrize("form", ["f64", "f32", "bf16x6"])
def test_maximum_n_against_the_diagonal_closed_form(form, torch_cuda):
    """n = 16384 (the largest the ABI accepts: 256 rotation stages, a 16384-long
    fused K loop) with Z = I, i.e. Phi = diag(w): then M_j is diagonal and Eq. 1
    is evaluated directly, b = (X^T D X)^-1 X^T D y with D = M_j^-1, in FP64."""
    torch = torch_cuda
    n, p, m, t = 16384, 4, 96, 8
    rng = np.random.default_rng(16384)
    w = rng.uniform(0.5, 2.0, n)
    xl = np.vstack([np.ones(n), rng.standard_normal((p - 2, n))])
    xr = rng.integers(0, 3, size=(m, n), dtype=np.uint8)
    y = rng.standard_normal((t, n))
    h2 = rng.uniform(0.1, 0.9, t)
    xf = xr.astype(np.float64)
    ref = np.empty((m, t, p))
    for j in range(t):
        d = 1.0 / (h2[j] * w + 1.0 - h2[j])
        a = xl * d                                   # (p-1) x n
        s = np.empty((m, p, p))
        s[:, :p - 1, :p - 1] = a @ xl.T
        s[:, :p - 1, p - 1] = (a @ xf.T).T
        s[:, p - 1, :p - 1] = s[:, :p - 1, p - 1]
        s[:, p - 1, p - 1] = (xf * xf) @ d
        r = np.empty((m, p))
        r[:, :p - 1] = a @ y[j]
        r[:, p - 1] = xf @ (d * y[j])
        ref[:, j] = np.linalg.solve(s, r[..., None])[..., 0]
    from paper_1210_7683_amd import gwas
    with gwas.Cohort(np.eye(n), w, xl, m, forms=(form,), max_traits=t) as c:
        c.rotate(0, torch.from_numpy(xr).cuda())
        b = c.solve(y, h2, form=form).cpu().numpy()
    assert np.isfinite(b).all()
    check_bound(b, ref, form, label="n=%d, Z = I" % n)


@pytest.fixture(scope="module")
def paper_m1e5(torch_cuda):
    """The paper-shape workload (n = 1000, p = 4, m = 1e5, t = 1000) resident on the GPU."""
    torch = torch_cuda
    w = synth.WORKLOADS["paper_m1e5"]
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    ev, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    c = gwas.Cohort(z, ev, xl, w.m, forms=ALL_FORMS)
    c.rotate(0, torch.from_numpy(xr).cuda())
    yd = torch.from_numpy(y).cuda()
    yield dict(w=w, phi=phi, xl=xl, y=y, h2=h2, c=c, yd=yd)
    c.close()


@pytest.mark.parametrize("form", FORMS)
def test_paper_shape_sampled_against_oracle(paper_m1e5, form, torch_cuda):
    d = paper_m1e5
    b = d["c"].solve(d["yd"], d["h2"], form=form)
    # six random traits (one O(n^3) factorisation each keeps the oracle to seconds),
    # 60 random SNPs each, plus the first and last SNP and trait of the grid
    rng = np.random.default_rng(11)
    traits = np.concatenate([[0, d["w"].t - 1], rng.choice(np.arange(1, d["w"].t - 1), 4, replace=False)])
    jj = np.repeat(traits, 62)
    ii = np.concatenate([np.concatenate([[0, d["w"].m - 1], rng.choice(d["w"].m, 60, replace=False)])
                         for _ in traits])
    got = b[torch_cuda.from_numpy(ii).cuda(), torch_cuda.from_numpy(jj).cuda()].cpu().numpy()
    uj, inv = np.unique(jj, return_inverse=True)
    ref = oracle.gls(d["phi"], d["xl"], synth.snp_columns(d["w"], ii), d["y"][uj], d["h2"][uj],
                     trait=inv)
    err = rel_err(got, ref)
    print("paper_m1e5 %s sampled %d: max %.3e median %.3e" % (form, err.size, err.max(), np.median(err)))
    assert err.max() <= TOL[form]
    assert bool(torch_cuda.isfinite(b).all())


@pytest.mark.parametrize("form", ["f32", "bf16x6", "bf16x3"])
def test_paper_shape_every_problem_against_the_fp64_form(paper_m1e5, form, torch_cuda):
    """All 10^8 problems of the paper-shape grid against the FP64 form, which the
    sampled test above holds to 1e-10 of the oracle: the bound must hold for the
    tail of the whole grid, not only for a sample."""
    d = paper_m1e5
    b64 = d["c"].solve(d["yd"], d["h2"], form="f64")
    b = d["c"].solve(d["yd"], d["h2"], form=form)
    mx, (i, j), e = grid_error_vs(b, b64)
    above = int((e > TOL[form] / 10).sum())
    print("paper_m1e5 %s every problem vs FP64 form: max %.3e at (%d, %d), %d above %.0e" % (
        form, mx, i, j, above, TOL[form] / 10))
    assert mx <= TOL[form] - 1e-10


def _checksum_numpy(a):
    """Sum over the 32-bit words w_k of (k + 1) w_k, modulo 2^64 (numpy wraps uint64)."""
    w = np.ascontiguousarray(a).reshape(-1).view(np.uint32).astype(np.uint64)
    return int((w * np.arange(1, w.size + 1, dtype=np.uint64)).sum(dtype=np.uint64))


@pytest.mark.parametrize("form", FORMS)
def test_streamed_slabs_match_resident_b_and_checksums(form, torch_cuda):
    """b streamed through the pinned ring equals, slab by slab, the b computed resident in HBM."""
    phi, xl, xr, y, h2 = synth.small(128, 4, 700, 45, seed=13)
    c = cohort(phi, xl, xr, forms=(form,), slab_snps=160, max_traits=16, ring_slots=3, host_threads=3)
    dev = c.solve(y, h2, form=form).cpu().numpy()
    seen = []

    def on_slab(info, arr):
        ref = dev[info["i0"]:info["i0"] + info["count"], info["j0"]:info["j0"] + info["tb"]]
        assert np.array_equal(arr, ref)
        assert info["checksum"] == _checksum_numpy(ref)
        seen.append((info["i0"], info["j0"]))

    sums = c.solve_stream(y, h2, form=form, on_slab=on_slab)
    assert len(sums) == len(seen) == 5 * 3              # 5 SNP slabs x 3 trait sub-blocks
    assert len(set(seen)) == len(seen)
    from paper_1210_7683_amd import gwas
    assert gwas.checksum(dev[:160, :16]) == _checksum_numpy(dev[:160, :16]) == sums[0]
    c.close()


def test_large_n_sampled_against_oracle(torch_cuda):
    """n = 4096 samples (a K loop four times the paper's, 128 stages of FP64 folds
    in the FP32 form), m = 1500, t = 8, every form; 300 sampled problems against
    the oracle (one dense Cholesky of each M_j)."""
    torch = torch_cuda
    n, p, m, t = 4096, 4, 1500, 8
    phi, xl, xr, y, h2 = synth.small(n, p, m, t, seed=4096, k=2 * n)
    rng = np.random.default_rng(1)
    ii = rng.choice(m, size=300, replace=False)
    jj = rng.integers(0, t, size=300)
    ref = oracle.gls(phi, xl, xr[ii], y, h2, trait=jj)
    w, z = np.linalg.eigh(phi)
    from paper_1210_7683_amd import gwas
    with gwas.Cohort(z, w, xl, m, forms=ALL_FORMS) as c:
        c.rotate(0, torch.from_numpy(xr).cuda())
        for form in FORMS:
            b = c.solve(y, h2, form=form)
            got = b[torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()].cpu().numpy()
            e = rel_err(got, ref)
            print("n=%d %s: relative max %.3e, median %.3e" % (n, form, e.max(), np.median(e)))
            assert bool(torch.isfinite(b).all())
            assert e.max() <= TOL[form]
