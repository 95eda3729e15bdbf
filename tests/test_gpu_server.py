"""The continuous-batching server: parity, alone-vs-mix identity, admission, cancellation.

Requests carry their own traits, heritabilities and covariate count p (a
prefix of the cohort's intercept-first covariates). Each result is checked
against the FP64 oracle (the FP64 form per problem at 1e-10), a request's b is
required to be bitwise the same when it runs alone and when it runs in a mix
with other requests, and, with the cohort's full covariate set, the same as
the direct solve of the same traits.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import ALL_FORMS, check_bound

pytestmark = pytest.mark.gpu

N, PMAX, M = 128, 8, 700


@pytest.fixture(scope="module")
def cohort_all():
    import torch
    assert torch.cuda.is_available()
    from paper_1210_7683_amd import gwas
    phi, xl, xr, _, _ = synth.small(N, PMAX, M, 1, seed=41)
    w, z = np.linalg.eigh(phi)
    c = gwas.Cohort(z, w, xl, M, forms=ALL_FORMS)
    c.rotate(0, xr)
    yield dict(c=c, phi=phi, xl=xl, xr=xr)
    c.close()


def _requests(seed, count, n=N):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        t = int(rng.choice([1, 3, 17, 40, 64]))
        p = int(rng.integers(2, PMAX + 1))
        out.append((rng.standard_normal((t, n)), rng.uniform(0.1, 0.9, t), p))
    return out


def _run(server, reqs, together, m=M):
    dt = np.float64 if server.form == "f64" else np.float32
    outs, tickets = [], []
    for y, h2, p in reqs:
        out = np.empty((m, y.shape[0], p), dtype=dt)
        tk = server.submit(y, h2, p, out=out)
        if not together:
            assert server.wait(tk, timeout=60)["state"] == "done"
        outs.append(out)
        tickets.append(tk)
    res = [server.wait(tk, timeout=60) for tk in tickets]
    assert all(r["state"] == "done" for r in res), res
    return outs, res


@pytest.mark.parametrize("form", ALL_FORMS)
def test_alone_equals_mix_and_matches_oracle(cohort_all, form):
    from paper_1210_7683_amd import gwas
    d = cohort_all
    reqs = _requests(1, 7)
    with gwas.Server(d["c"], form=form, max_slots=4, item_problems=6000, max_traits=64) as srv:
        alone, _ = _run(srv, reqs, together=False)
        st0 = srv.stats()
        mix, res = _run(srv, reqs, together=True)
        st1 = srv.stats()
    for a, b in zip(alone, mix):
        assert np.array_equal(a, b)
    # the mix was batched: its grouped launches carried more than one slab each on average
    items, rounds = st1["items"] - st0["items"], st1["rounds"] - st0["rounds"]
    print("%s mix: %d slabs in %d launches" % (form, items, rounds))
    assert items > rounds
    # overlap: in the mix, some request was admitted before another finished
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    assert any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))
    for (y, h2, p), b in zip(reqs, alone):
        ref = oracle.gls_grid(d["phi"], d["xl"][: p - 1], d["xr"], y, h2)
        check_bound(b, ref, form, label="served p=%d t=%d" % (p, y.shape[0]))


@pytest.mark.parametrize("form", ALL_FORMS)
def test_served_b_equals_the_direct_solve(cohort_all, form):
    """A request with the cohort's full covariate set gets, bitwise, the b that
    gwas_solve computes for the same traits (the same per-problem tile
    arithmetic: K order, MFMA products and FP64 folds), alone and in a mix."""
    from paper_1210_7683_amd import gwas
    d = cohort_all
    rng = np.random.default_rng(77)
    reqs = [(rng.standard_normal((t, N)), rng.uniform(0.1, 0.9, t), PMAX) for t in (5, 17, 40)]
    with gwas.Server(d["c"], form=form, max_slots=3, item_problems=6000, max_traits=64) as srv:
        served, _ = _run(srv, reqs, together=True)
    for (y, h2, _), b in zip(reqs, served):
        direct = d["c"].solve(y, h2, form=form).cpu().numpy()
        diff = np.abs(direct.astype(np.float64) - b).max()
        assert np.array_equal(direct, b), (form, y.shape[0], diff)


@pytest.fixture(scope="module")
def cohort_n1000():
    """The serving workload's cohort shape, n = 1000 with the intercept and six
    covariates (p up to 8), on 3000 SNPs, every form resident."""
    import torch
    assert torch.cuda.is_available()
    from paper_1210_7683_amd import gwas
    phi, xl, xr, _, _ = synth.small(1000, PMAX, 3000, 1, seed=1000)
    w, z = np.linalg.eigh(phi)
    c = gwas.Cohort(z, w, xl, 3000, forms=ALL_FORMS)
    c.rotate(0, torch.from_numpy(xr).cuda())
    torch.cuda.synchronize()
    yield dict(c=c, phi=phi, xl=xl, xr=xr)
    c.close()


def test_serving_at_the_cohort_shape_against_oracle(cohort_n1000):
    """n = 1000, requests at every p = 2..8 with trait counts 1 to 100, all in
    one mix per form: a sample of each request's problems (three traits, 40
    SNPs each, including the first and last SNP) against the oracle, the FP64
    form per problem at 1e-10 and the reduced forms at their bounds."""
    from paper_1210_7683_amd import gwas
    d = cohort_n1000
    m = d["xr"].shape[0]
    rng = np.random.default_rng(1000)
    ts = [1, 100, 3, 17, 64, 9, 33]
    reqs = [(rng.standard_normal((t, 1000)), rng.uniform(0.1, 0.9, t), p) for p, t in zip(range(2, 9), ts)]
    picks, refs = [], []
    for y, h2, p in reqs:
        tj = rng.choice(y.shape[0], size=min(3, y.shape[0]), replace=False)
        ii = np.concatenate([[0, m - 1], rng.choice(np.arange(1, m - 1), 38, replace=False)])
        jj = np.repeat(tj, ii.size)
        iii = np.tile(ii, tj.size)
        uj, inv = np.unique(jj, return_inverse=True)
        refs.append(oracle.gls(d["phi"], d["xl"][: p - 1], d["xr"][iii], y[uj], h2[uj], trait=inv))
        picks.append((iii, jj))
    for form in ALL_FORMS:
        with gwas.Server(d["c"], form=form, max_slots=8, item_problems=100_000, max_traits=128) as srv:
            outs, _ = _run(srv, reqs, together=True, m=m)
        for (y, h2, p), b, (iii, jj), ref in zip(reqs, outs, picks, refs):
            check_bound(b[iii, jj], ref, form, label="n=1000 served p=%d t=%d" % (p, y.shape[0]))
            assert np.isfinite(b).all()


def test_ring_checksums(cohort_all):
    from paper_1210_7683_amd import gwas
    d = cohort_all
    reqs = _requests(2, 4)
    with gwas.Server(d["c"], form="f32", max_slots=3, item_problems=5000, max_traits=64) as srv:
        ref, _ = _run(srv, reqs, together=False)
        tickets = [srv.submit(y, h2, p) for y, h2, p in reqs]
        res = [srv.wait(tk, timeout=60) for tk in tickets]
    for (y, h2, p), b, r in zip(reqs, ref, res):
        t = y.shape[0]
        slab = min(M, max(256, 5000 // t // 256 * 256))
        expect = 0
        for s0 in range(0, M, slab):
            expect = (expect + gwas.checksum(b[s0:s0 + slab])) % (1 << 64)
        assert r["state"] == "done" and r["slabs"] == -(-M // slab)
        assert r["checksum"] == expect


def test_admission_by_memory_serialises_requests(cohort_all):
    from paper_1210_7683_amd import gwas
    d = cohort_all
    rng = np.random.default_rng(3)
    reqs = [(rng.standard_normal((64, N)), rng.uniform(0.1, 0.9, 64), 4) for _ in range(4)]
    # each request holds ~1.4 MB (traits, panels, factors, four 256 KB b stages):
    # a 1.6 MB budget admits one at a time although 8 slots are free
    with gwas.Server(d["c"], form="f32", max_slots=8, hbm_budget=1600 << 10, item_problems=6000,
                     max_traits=64) as srv:
        outs, res = _run(srv, reqs, together=True)
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    for k in range(len(spans) - 1):
        assert spans[k + 1][0] >= spans[k][1]


def test_cancel_and_errors(cohort_all):
    from paper_1210_7683_amd import gwas
    d = cohort_all
    y = np.random.default_rng(0).standard_normal((64, N))
    h2 = np.full(64, 0.5)
    with gwas.Server(d["c"], form="f32", max_slots=1, item_problems=2000, max_traits=64) as srv:
        first = srv.submit(y, h2, 8)
        queued = srv.submit(y, h2, 8)
        srv.cancel(queued)
        srv.cancel(first)
        assert srv.wait(queued, timeout=60)["state"] == "cancelled"
        assert srv.wait(first, timeout=60)["state"] in ("cancelled", "done")
        for bad in [dict(p=1), dict(p=PMAX + 1), dict(m=M + 1), dict(i0=M)]:
            args = dict(p=4)
            args.update(bad)
            with pytest.raises(gwas.GwasError):
                srv.submit(y, h2, **args)
        with pytest.raises(gwas.GwasError):
            srv.submit(y, np.full(64, 1.5), 4)
        with pytest.raises(gwas.GwasError):
            srv.poll(12345)
    w, z = np.linalg.eigh(d["phi"])
    with gwas.Cohort(z, w, d["xl"], 16, forms=("f32",)) as c32:
        for form in ("f64", "bf16x3", "bf16x6"):
            with pytest.raises(gwas.GwasError, match="not resident"):
                gwas.Server(c32, form=form, item_problems=2000, max_traits=64)
    with gwas.Server(d["c"], form="f32", hbm_budget=1 << 16, item_problems=2000, max_traits=64) as small:
        with pytest.raises(gwas.GwasError):       # can never fit the budget
            small.submit(y, h2, 4)
