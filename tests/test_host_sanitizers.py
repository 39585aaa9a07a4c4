"""Host-side table construction under AddressSanitizer and UBSan (CPU only).

The grid, blockwise Hilbert ordering, row neighbour table, projector
supports, per-row KB entries and block atom lists are built by host C++
(paper_2303_00790_amd/csrc/host_grid.cpp).  tests/host_sanitize_main.cpp
drives them on small clusters (both orderings, three spacings) with the host
compiler's address and undefined-behaviour sanitizers and checks their
invariants: every stencil offset that leaves a block lands in the block its
face table names, the blocks' inside masks are exactly the inside rows, padding
rows have no neighbours, the per-row projector entries are the exact transpose of the
per-atom supports, each block's atom list holds exactly the atoms with an entry
in its rows, and every entry's slot names its own atom.  Any sanitizer report
fails the test.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2303_00790_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_host_tables_clean_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("host C++ compiler or HIP headers not available")
    exe = tmp_path / "host_san"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-I", CSRC, "-I", os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__", os.path.join(HERE, "host_sanitize_main.cpp"), os.path.join(CSRC, "host_grid.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ok" in r.stdout.split()
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
