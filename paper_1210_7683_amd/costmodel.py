"""Operation and byte counts of the GLS grid (host-side bookkeeping for measurement).

Counts follow the paper's cost column of Algorithm 5 and its I/O analysis
(Section 4): the per-problem work of the inner loop is (5 + 2(p-1)) n flops
(Section 4.2, the constraint on tb); the rotation GEMMs cost 2 n^2 per column
(Algorithm 5, preloop); a tile's I/O is (mb n + mb tb p) elements.

The GPU kernel evaluates the inner loop as p+1 contractions of length n per
(SNP, trait) pair, so its algorithmic count is 2 (p+1) n flops per problem;
both conventions are reported.
"""
from __future__ import annotations


def flops_per_gls_paper(n: int, p: int) -> int:
    """Inner-loop flops per (SNP, trait) problem as the paper counts them."""
    return (5 + 2 * (p - 1)) * n


def flops_per_gls_contraction(n: int, p: int) -> int:
    """Flops of the p+1 length-n contractions per problem (the fused kernel's MFMA work)."""
    return 2 * (p + 1) * n


def rotation_flops(n: int, cols: int) -> int:
    """Z^T X for an n x cols block (Algorithm 5, preloop GEMMs)."""
    return 2 * n * n * cols


def grid_flops_paper(n: int, p: int, m: int, t: int) -> int:
    return flops_per_gls_paper(n, p) * m * t


def naive_stream_bytes(n: int, m: int, t: int, itemsize: int = 8) -> int:
    """Traffic of reloading the whole X_R once per trait (the naive scheme of Section 4)."""
    return n * m * t * itemsize


def output_bytes(m: int, t: int, p: int, itemsize: int) -> int:
    return m * t * p * itemsize


def eq_nb_holds(n: int, gemm_flops_per_s: float, itemsize: int, io_bytes_per_s: float) -> bool:
    """Overlap condition of the preloop stream: n / F > sizeof / BW (Section 4.1)."""
    return n / gemm_flops_per_s > itemsize / io_bytes_per_s


def eq_tb_holds(tb: int, n: int, p: int, tile_flops_per_s: float, itemsize: int,
                io_bytes_per_s: float) -> bool:
    """Overlap condition of a tile (Section 4.2), divided through by mb:
    tb (5 + 2(p-1)) n / F > (n + tb p) sizeof / BW."""
    return tb * flops_per_gls_paper(n, p) / tile_flops_per_s > \
        (n + tb * p) * itemsize / io_bytes_per_s


def min_tb(n: int, p: int, tile_flops_per_s: float, itemsize: int, io_bytes_per_s: float,
           limit: int = 1 << 30) -> int | None:
    """Smallest trait-tile width tb for which a tile's compute hides its I/O."""
    tb = 1
    while tb <= limit:
        if eq_tb_holds(tb, n, p, tile_flops_per_s, itemsize, io_bytes_per_s):
            return tb
        tb *= 2
    else:
        return None


def min_tb_exact(n: int, p: int, tile_flops_per_s: float, itemsize: int,
                 io_bytes_per_s: float) -> int | None:
    """Closed form of the smallest integer tb satisfying the tile overlap condition."""
    a = flops_per_gls_paper(n, p) / tile_flops_per_s - p * itemsize / io_bytes_per_s
    if a <= 0:
        return None
    c = n * itemsize / io_bytes_per_s
    tb = int(c // a) + 1
    while tb > 1 and eq_tb_holds(tb - 1, n, p, tile_flops_per_s, itemsize, io_bytes_per_s):
        tb -= 1
    return tb


def tile_ratio(tb: int, n: int, p: int) -> float:
    """Compute-to-transfer ratio of a tile per SNP, tb p n / (n + tb p), up to the O() constant."""
    return tb * p * n / (n + tb * p)
