"""Host check of the row hash lookup the samplers' adjacency tests use
(csrc/rowhash.hpp): compiled for the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer against a table of exactly the size preparation
allocates, compared with std::binary_search on heavy-tailed rows (empty
rows, single slots, one long row, keys shared with neighbouring rows and
with the padding after the last row)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rowhash_exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("rowhash") / "rowhash_check")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", os.path.join(HERE, "rowhash_check.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("seed,slots,queries", [(1, 1, 1000), (2, 5, 5000), (3, 64, 20000), (4, 1000, 50000),
                                                (5, 100000, 200000), (7, 20000, 200000),
                                                (6, 2000000, 200000)])
def test_rowhash_matches_binary_search(rowhash_exe, seed, slots, queries):
    r = subprocess.run([rowhash_exe, str(seed), str(slots), str(queries)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches=0" in r.stdout
