"""Precision study at paper shape: n = 1000, p = 4, m = 1,000,000 SNPs, t = 1,000 traits.

The full grid (10^9 problems) is solved on the GPU in each form; a seeded
uniform sample of 10,000 (SNP, trait) problems is solved by the FP64 oracle
(dense Cholesky of each M_j) and compared problem by problem. The statistics
(max, p99.99 and median relative error, and the scaled error) are printed as
one JSON line per form; the bounds are the stated ones. Every problem of the
reduced forms' grids is then compared with the FP64 form's grid (held to 1e-10
of the oracle by the sample), so the bound is checked on the whole tail.
"""
import json
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import ALL_FORMS, TOL, grid_error_vs, rel_err, scaled_err

pytestmark = pytest.mark.gpu


def test_precision_study_paper_m1e6():
    import torch

    from paper_1210_7683_amd import gwas

    assert torch.cuda.is_available()
    w = synth.WORKLOADS["paper_m1e6"]
    t0 = time.perf_counter()
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    ev, z = np.linalg.eigh(phi)
    print("inputs %.1f s" % (time.perf_counter() - t0), flush=True)
    ii, jj = synth.sample_problems(w, 10_000)
    uj, inv = np.unique(jj, return_inverse=True)
    t0 = time.perf_counter()
    ref = oracle.gls(phi, xl, xr[ii], y[uj], h2[uj], trait=inv)
    print("oracle: %d problems over %d traits in %.1f s" % (ii.size, uj.size, time.perf_counter() - t0),
          flush=True)
    ti, tj = torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()
    xd = torch.from_numpy(xr).cuda()
    yd = torch.from_numpy(y).cuda()
    rng = np.random.default_rng(5)
    i1 = np.sort(rng.choice(w.m, size=10_000, replace=False))
    ref1 = oracle.gls(phi, xl, xr[i1], y[:1], h2[:1], trait=np.zeros(i1.size, dtype=np.int64))
    t1 = torch.from_numpy(i1).cuda()
    # one cohort per form, as a run of one form holds it: the rotation then
    # uses all six Z digits for the FP64 form and the leading four otherwise
    assert ALL_FORMS[0] == "f64"
    b64 = None
    for form in ALL_FORMS:
        with gwas.Cohort(z, ev, xl, w.m, forms=(form,)) as c:
            c.rotate(0, xd)
            b = c.solve(yd, h2, form=form)
            got = b[ti, tj].cpu().numpy()
            finite = bool(torch.isfinite(b).all())
            if form == "f64":
                b64 = b
            else:
                mx, (gi, gj), eg = grid_error_vs(b, b64)
                strided = eg.reshape(-1)[::97]
                grid = {"form": form, "vs": "f64 form", "problems": int(eg.numel()), "rel_max": mx,
                        "at": [gi, gj], "above_bound": int((eg > TOL[form]).sum()),
                        "rel_p9999_strided": float(torch.quantile(strided, 0.9999)),
                        "rel_median_strided": float(strided.median())}
                print("PRECISION_GRID " + json.dumps(grid), flush=True)
                del eg, strided
                assert mx <= TOL[form] - 1e-10, grid
            del b
            torch.cuda.empty_cache()
            e = rel_err(got, ref)
            # the sample holds ~10 problems per trait: scale by the sample's median ||b||
            s = scaled_err(got[None], ref[None], trait_axis=0)[0]
            stats = {"form": form, "problems": int(e.size), "rel_max": float(e.max()),
                     "rel_p9999": float(np.quantile(e, 0.9999)), "rel_median": float(np.median(e)),
                     "scaled_max": float(s.max()), "all_finite": finite}
            print("PRECISION " + json.dumps(stats), flush=True)
            assert finite
            assert e.max() <= TOL[form], stats
            if form not in ("f64", "f32"):
                continue
            # single-trait calls (the dot-product kernel in the FP64 and FP32 forms)
            c.reset_stats()
            b = c.solve(yd[:1], h2[:1], form=form)
            assert c.stats()["dot_launches"] == 1
            got = b[t1, 0].cpu().numpy()
            finite = bool(torch.isfinite(b).all())
            del b
            e = rel_err(got, ref1)
            stats = {"form": form, "t": 1, "problems": int(e.size), "rel_max": float(e.max()),
                     "rel_p9999": float(np.quantile(e, 0.9999)), "rel_median": float(np.median(e)),
                     "all_finite": finite}
            print("PRECISION " + json.dumps(stats), flush=True)
            assert finite
            assert e.max() <= TOL[form], stats
