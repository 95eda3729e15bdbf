"""The serving loop's first-fit arena (csrc/arena.h), checked on the host.

tests/arena_check.cpp drives the arena through random alloc/release sequences
against a granule model (disjoint live blocks, a coalesced free list covering
exactly the rest, first fit); it is compiled here with g++, with the address
and undefined-behaviour sanitizers where the toolchain has them.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1210_7683_amd", "csrc")


def _build(tmp_path, flags):
    exe = str(tmp_path / "arena_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-I" + CSRC] + flags + [os.path.join(HERE, "arena_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return exe if r.returncode == 0 else None, r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_arena_first_fit_and_coalescing(tmp_path):
    exe, err = _build(tmp_path, ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"])
    if exe is None:   # no sanitizer runtime: the plain build still checks the invariants
        exe, err = _build(tmp_path, [])
    assert exe is not None, err
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failed checks" in r.stdout
