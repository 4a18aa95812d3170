"""Host check of the row search index the sampling kernels use
(csrc/ladder.hpp): compiled for the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer, compared with std::binary_search on random
heavy-tailed rows, including one row longer than 32^4 slots."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ladder_exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("ladder") / "ladder_check")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", os.path.join(HERE, "ladder_check.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("seed,slots,queries", [(7, 20, 5000), (8, 32, 5000), (9, 33, 5000), (2, 1000, 50000),
                                                (11, 32769, 100000), (3, 100000, 100000), (4, 3000000, 200000),
                                                (5, 40000000, 100000)])
def test_ladder_matches_binary_search(ladder_exe, seed, slots, queries):
    r = subprocess.run([ladder_exe, str(seed), str(slots), str(queries)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches=0" in r.stdout
