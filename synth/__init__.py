"""Seeded synthetic inputs shaped like the paper's GWAS workloads.

This module draws inputs only. It holds none of the method's arithmetic and is
shared by the CPU oracle's tests and by the GPU path's tests and benchmark.

Shapes follow the problem statement (Section 2 and Section 3.3 of the paper):
n samples, m SNPs, t traits, p columns per design matrix X_i = [X_L | x_i].

Recipe (the same for every workload):
  * minor-allele frequency maf ~ U(0.05, 0.5) per SNP;
  * genotype = Bernoulli(maf) + Bernoulli(maf), i.e. Binomial(2, maf), uint8;
    a column whose n values are all equal (monomorphic) is redrawn, since the
    paper assumes every X_i has full rank;
  * kinship Phi = G G^T / k + 1e-3 I from an n x k genotype matrix G drawn the
    same way and standardized column-wise with its generating maf,
    (g - 2 maf) / sqrt(2 maf (1 - maf));
  * X_L = [1 | N(0,1) ...], n x (p-1), column-major (each column contiguous);
  * Y ~ N(0,1), trait-major (each trait's n values contiguous);
  * h2 ~ U(0.1, 0.9) per trait.

Seeds: numpy SeedSequence(12107683), one child per workload; inside a workload
the SNP axis is drawn in blocks of 65,536 SNPs and the trait axis in blocks of
1,024 traits, each block from its own child, so any block can be regenerated
alone (the oracle's sampled checks at full size depend on this).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = 12107683
SNP_BLOCK = 65536
TRAIT_BLOCK = 1024

# child indices inside a workload's SeedSequence
_K_KIN, _K_XL, _K_XR, _K_Y, _K_H2, _K_ARRIVAL, _K_SAMPLE, _K_REQ = range(8)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int          # child of the root SeedSequence
    n: int              # samples
    p: int              # columns of X_i (intercept + covariates + 1 SNP)
    m: int              # SNPs
    t: int              # traits
    k: int              # SNPs used to build the kinship matrix

    @property
    def problems(self) -> int:
        return self.m * self.t


# The seven workloads: tiny FP64 check; paper shape (n=1000, p=4) at m=1e5 and
# m=1e6; a streamed 1e6 x 1e4 grid; a resident 1e6-SNP cohort for serving; the
# single-trait case (t = 1) of the same cohort shape; and 4e6 SNPs streamed
# from host memory through a 2^20-SNP store.
WORKLOADS = {
    "tiny": Workload("tiny", 0, n=128, p=4, m=512, t=8, k=1000),
    "paper_m1e5": Workload("paper_m1e5", 1, n=1000, p=4, m=100_000, t=1000, k=5000),
    "paper_m1e6": Workload("paper_m1e6", 2, n=1000, p=4, m=1_000_000, t=1000, k=5000),
    "stream_m1e6_t1e4": Workload("stream_m1e6_t1e4", 3, n=1000, p=4, m=1_000_000, t=10_000, k=5000),
    "serve_m1e6": Workload("serve_m1e6", 4, n=1000, p=8, m=1_000_000, t=512, k=5000),
    "single_trait_m1e6": Workload("single_trait_m1e6", 5, n=1000, p=4, m=1_000_000, t=1, k=5000),
    "snp_stream_m4e6_t100": Workload("snp_stream_m4e6_t100", 6, n=1000, p=4, m=4_000_000, t=100, k=5000),
}


def _child(ss: np.random.SeedSequence, *key: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(entropy=ss.entropy, spawn_key=tuple(ss.spawn_key) + tuple(key))


def workload_seed(w: Workload | str) -> np.random.SeedSequence:
    if isinstance(w, str):
        w = WORKLOADS[w]
    return _child(np.random.SeedSequence(ROOT_SEED), w.index)


def _genotypes(rng: np.random.Generator, n: int, cols: int) -> tuple[np.ndarray, np.ndarray]:
    """Binomial(2, maf) genotypes, one column (n values, contiguous) per SNP.

    Returns (g [cols][n] uint8, maf [cols] float64). Monomorphic columns are
    redrawn with the same generator until none remains.
    """
    maf = rng.uniform(0.05, 0.5, size=cols)
    mf = maf.astype(np.float32)[:, None]
    g = (rng.random((cols, n), dtype=np.float32) < mf).astype(np.uint8)
    g += (rng.random((cols, n), dtype=np.float32) < mf).astype(np.uint8)
    while True:
        bad = np.flatnonzero((g == g[:, :1]).all(axis=1))
        if bad.size == 0:
            break
        mb = mf[bad]
        r = (rng.random((bad.size, n), dtype=np.float32) < mb).astype(np.uint8)
        r += (rng.random((bad.size, n), dtype=np.float32) < mb).astype(np.uint8)
        g[bad] = r
    return g, maf


def kinship(w: Workload | str) -> np.ndarray:
    """Phi = G G^T / k + 1e-3 I, n x n symmetric positive definite."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.default_rng(_child(workload_seed(w), _K_KIN))
    g, maf = _genotypes(rng, w.n, w.k)                      # [k][n]
    gs = (g.astype(np.float64) - 2.0 * maf[:, None]) / np.sqrt(2.0 * maf * (1.0 - maf))[:, None]
    phi = gs.T @ gs / w.k
    phi = 0.5 * (phi + phi.T)
    phi[np.diag_indices(w.n)] += 1e-3
    return phi


def covariates(w: Workload | str, p: int | None = None) -> np.ndarray:
    """X_L: [(p-1)][n] float64 (column-major n x (p-1)); column 0 is all ones."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    p = w.p if p is None else p
    rng = np.random.default_rng(_child(workload_seed(w), _K_XL))
    pool = rng.standard_normal((19, w.n))    # the first p-2 are used; p <= 20
    xl = np.empty((p - 1, w.n))
    xl[0] = 1.0
    xl[1:] = pool[: p - 2]
    return xl


def snps(w: Workload | str, m0: int = 0, mb: int | None = None) -> np.ndarray:
    """Genotypes of SNPs [m0, m0+mb): [mb][n] uint8 (n x mb column-major)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    mb = w.m - m0 if mb is None else mb
    if m0 < 0 or mb < 0 or m0 + mb > w.m:
        raise ValueError("SNP range outside the workload")
    out = np.empty((mb, w.n), dtype=np.uint8)
    root = _child(workload_seed(w), _K_XR)
    b0, b1 = m0 // SNP_BLOCK, (m0 + mb + SNP_BLOCK - 1) // SNP_BLOCK
    for b in range(b0, b1):
        lo = b * SNP_BLOCK
        cols = min(SNP_BLOCK, w.m - lo)
        g, _ = _genotypes(np.random.default_rng(_child(root, b)), w.n, cols)
        s0, s1 = max(m0, lo), min(m0 + mb, lo + cols)
        out[s0 - m0 : s1 - m0] = g[s0 - lo : s1 - lo]
    return out


def snp_columns(w: Workload | str, idx: np.ndarray) -> np.ndarray:
    """Genotypes of the SNPs listed in idx: [len(idx)][n] uint8."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty((idx.size, w.n), dtype=np.uint8)
    for b in np.unique(idx // SNP_BLOCK):
        sel = np.flatnonzero(idx // SNP_BLOCK == b)
        blk = snps(w, int(b) * SNP_BLOCK, min(SNP_BLOCK, w.m - int(b) * SNP_BLOCK))
        out[sel] = blk[idx[sel] - int(b) * SNP_BLOCK]
    return out


def _trait_block(w: Workload, b: int) -> tuple[np.ndarray, np.ndarray]:
    cols = min(TRAIT_BLOCK, w.t - b * TRAIT_BLOCK)
    ss = workload_seed(w)
    y = np.random.default_rng(_child(ss, _K_Y, b)).standard_normal((cols, w.n))
    h2 = np.random.default_rng(_child(ss, _K_H2, b)).uniform(0.1, 0.9, size=cols)
    return y, h2


def traits(w: Workload | str, t0: int = 0, tb: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Traits [t0, t0+tb): (Y [tb][n] float64, h2 [tb] float64)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    tb = w.t - t0 if tb is None else tb
    if t0 < 0 or tb < 0 or t0 + tb > w.t:
        raise ValueError("trait range outside the workload")
    y = np.empty((tb, w.n))
    h2 = np.empty(tb)
    for b in range(t0 // TRAIT_BLOCK, (t0 + tb + TRAIT_BLOCK - 1) // TRAIT_BLOCK):
        yb, hb = _trait_block(w, b)
        lo = b * TRAIT_BLOCK
        s0, s1 = max(t0, lo), min(t0 + tb, lo + yb.shape[0])
        y[s0 - t0 : s1 - t0] = yb[s0 - lo : s1 - lo]
        h2[s0 - t0 : s1 - t0] = hb[s0 - lo : s1 - lo]
    return y, h2


def sample_problems(w: Workload | str, count: int, salt: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """A seeded uniform sample of distinct (SNP, trait) pairs, sorted by trait."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.default_rng(_child(workload_seed(w), _K_SAMPLE, salt))
    count = min(count, w.m * w.t)
    flat = rng.choice(w.m * w.t, size=count, replace=False)
    i, j = flat // w.t, flat % w.t
    order = np.lexsort((i, j))
    return i[order].astype(np.int64), j[order].astype(np.int64)


@dataclasses.dataclass
class Request:
    """One serving request: a trait block with its own h2 and covariate count."""
    arrival_s: float
    p: int
    y: np.ndarray        # [t][n]
    h2: np.ndarray       # [t]


def requests(w: Workload | str, count: int, rate_hz: float, salt: int = 0,
             t_max: int = 512) -> list[Request]:
    """Poisson arrivals at rate_hz; t = clip(round(exp(U(0, ln t_max))), 1, t_max);
    p - 1 ~ U{1..7}; Y ~ N(0,1); h2 ~ U(0.1, 0.9)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.default_rng(_child(workload_seed(w), _K_REQ, salt))
    out, now = [], 0.0
    for _ in range(count):
        now += rng.exponential(1.0 / rate_hz) if rate_hz > 0 else 0.0
        t = int(min(t_max, max(1, round(math.exp(rng.uniform(0.0, math.log(t_max)))))))
        p = int(rng.integers(1, 8)) + 1
        out.append(Request(now, p, rng.standard_normal((t, w.n)), rng.uniform(0.1, 0.9, size=t)))
    return out


def small(n: int, p: int, m: int, t: int, seed: int, k: int | None = None):
    """A small ad-hoc workload with the same recipe: (Phi, X_L, X_R u8, Y, h2)."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 99, seed]))
    k = 4 * n if k is None else k
    g, maf = _genotypes(rng, n, k)
    gs = (g.astype(np.float64) - 2.0 * maf[:, None]) / np.sqrt(2.0 * maf * (1.0 - maf))[:, None]
    phi = gs.T @ gs / k
    phi = 0.5 * (phi + phi.T)
    phi[np.diag_indices(n)] += 1e-3
    xl = np.empty((p - 1, n))
    xl[0] = 1.0
    xl[1:] = rng.standard_normal((p - 2, n))
    xr, _ = _genotypes(rng, n, m)
    y = rng.standard_normal((t, n))
    h2 = rng.uniform(0.1, 0.9, size=t)
    return phi, xl, xr, y, h2
