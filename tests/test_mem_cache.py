"""Host checks of the library's device memory cache (csrc/lrx_cache.h).

The cache is a template over the mapper; tests/native/cache_check.cpp drives
it with a fake mapper (address ranges without memory) through random
allocation sequences, checking after each batch of steps that blocks tile
their segments, neighbouring free blocks are merged, live blocks are
disjoint, aligned and hold their requests, and the byte counts match; then
reuse without new mappings, the out-of-memory path (unmap idle segments,
map again) and the separation of small and large requests.  Built with g++,
under AddressSanitizer and UBSan when the toolchain has them.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2412_11081_amd", "csrc")
SRC = os.path.join(HERE, "native", "cache_check.cpp")


def _build(tmp_path, flags):
    exe = str(tmp_path / "cache_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-I", CSRC, *flags, "-o", exe, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return exe if r.returncode == 0 else None, r.stderr


def test_block_cache_invariants(tmp_path):
    exe, err = _build(tmp_path, ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"])
    if exe is None:
        exe, err = _build(tmp_path, [])
    assert exe is not None, err
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
