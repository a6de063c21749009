"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The basis-table builder (csrc/tables.cpp: the 1-D rules, the 1-D factor tables and their
derivatives, the collocation matrices, the index maps) is plain host C++.  It is built here with
g++ and both sanitizers, without recovery, together with tests/native/tables_sanitized.cpp,
which builds every shape at every order the builder accepts and reads every table in full.  No
GPU code is involved: the HIP headers are only parsed for their declarations.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_20917_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM_INC, "hip")),
                    reason="needs g++ and the HIP headers")
def test_table_builder_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "tables_sanitized")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           os.path.join(ROOT, "tests", "native", "tables_sanitized.cpp"), os.path.join(CSRC, "tables.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    # verify_asan_link_order=0: a library the environment preloads may come before the ASan runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
