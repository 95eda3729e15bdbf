"""GLS grid of multi-trait GWAS on one MI355X (gfx950).

The compute path is the C-ABI library libgwas.so (HIP kernels for gfx950);
`paper_1210_7683_amd.gwas` is its thin ctypes binding. Importing this package
does not load the library; the binding does, and raises if it is missing.
"""
__all__ = ["costmodel", "gwas"]
