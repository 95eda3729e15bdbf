"""The C-ABI library loads and exports every function include/gwas.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(gwas_[a-z0-9_]+)\s*\(",
                            text, flags=re.M)
    return names


def test_header_declares_the_core_calls():
    names = set(declared_functions())
    for core in ["gwas_setup", "gwas_rotate", "gwas_solve", "gwas_stats", "gwas_destroy",
                 "gwas_last_error"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1210_7683_amd import gwas
    if not os.path.exists(gwas.LIB_PATH):
        pytest.fail("libgwas.so is not built; run python -m paper_1210_7683_amd.build")
    lib = ctypes.CDLL(gwas.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    gwas.load()   # argtypes for every bound symbol resolve


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    from paper_1210_7683_amd import gwas
    monkeypatch.setattr(gwas, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gwas, "_lib", None)
    with pytest.raises(ImportError):
        gwas.load()


@pytest.mark.parametrize("bad", [1, 3, 4])
def test_setup_rejects_fold_intervals_other_than_0_and_2(bad):
    """Option checks run before any device call, so this needs no GPU."""
    import numpy as np

    from paper_1210_7683_amd import gwas
    if not os.path.exists(gwas.LIB_PATH):
        pytest.fail("libgwas.so is not built; run python -m paper_1210_7683_amd.build")
    n = 8
    z = np.eye(n)
    w = np.ones(n)
    xl = np.ones((1, n))
    with pytest.raises(gwas.GwasError, match="f32_flush"):
        gwas.Cohort(z, w, xl, 4, forms=("f32",), f32_flush=bad)


@pytest.mark.parametrize("bad", [-256, 100, 257])
def test_setup_rejects_genotype_chunks_not_a_multiple_of_256(bad):
    """geno_chunk_snps is checked with the other options, before any device call."""
    import numpy as np

    from paper_1210_7683_amd import gwas
    if not os.path.exists(gwas.LIB_PATH):
        pytest.fail("libgwas.so is not built; run python -m paper_1210_7683_amd.build")
    n = 8
    with pytest.raises(gwas.GwasError, match="geno_chunk_snps"):
        gwas.Cohort(np.eye(n), np.ones(n), np.ones((1, n)), 4, forms=("f32",), geno_chunk_snps=bad)


@pytest.mark.parametrize("n", [0, -3, 16385])
def test_eigh_rejects_sizes_out_of_range(n):
    """gwas_eigh checks n before it opens the solver or touches a device."""
    import numpy as np

    from paper_1210_7683_amd import gwas
    lib = gwas.load()
    z = np.zeros(4)
    w = np.zeros(2)
    st = lib.gwas_eigh(n, z.ctypes.data, z.ctypes.data, w.ctypes.data, 0, None)
    assert st == gwas.EINVAL
    assert "outside" in lib.gwas_last_error().decode()


def test_eigh_rejects_null_pointers():
    import numpy as np

    from paper_1210_7683_amd import gwas
    lib = gwas.load()
    w = np.zeros(2)
    assert lib.gwas_eigh(2, None, None, w.ctypes.data, 0, None) == gwas.EINVAL
