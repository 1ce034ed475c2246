"""AddressSanitizer / UndefinedBehaviorSanitizer build of libfpo's host code
(fpo_host.cpp: tree build, union, pruning, coarse occupancy, basis, cameras,
argument validation) and of the FP64 oracle (fpo_oracle.c, including its
threaded render, gradient and bake), driven by tests/native/sanitize_host.cpp.
Host compilers only (g++ / gcc); no device code is built or run."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INC = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC),
                    reason="needs g++ and the ROCm headers")
def test_host_code_and_oracle_under_asan_ubsan(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2202_08614_amd", "csrc"),
           "-I", ROCM_INC, "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src, cc, extra in (("oracle/fpo_oracle.c", "gcc", ["-std=gnu11"]),
                           ("paper_2202_08614_amd/csrc/fpo_host.cpp", "g++", ["-std=c++17", *inc]),
                           ("tests/native/sanitize_host.cpp", "g++", ["-std=c++17", *inc])):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([cc, *SAN, *extra, "-c", os.path.join(ROOT, src), "-o", obj], check=True,
                       capture_output=True, text=True)
        objs.append(obj)
    exe = str(tmp_path / "sanitize_host")
    subprocess.run(["g++", *SAN, *objs, "-o", exe, f"-L{ROCM_LIB}", f"-Wl,-rpath,{ROCM_LIB}", "-lamdhip64",
                    "-lrocprofiler-sdk-roctx", "-lpthread", "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "sanitize_host ok" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
