"""The library's host-only code (MBR schedule, GPS ordering, SAO and RANSAC
on host threads) and the C oracle, built with AddressSanitizer and
UndefinedBehaviorSanitizer by g++/gcc and run on seeded valid and invalid
inputs (tests/sanitize/host_checks.cpp).  CPU only; no HIP code is built."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_22089_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs g++ and gcc")
def test_host_code_and_oracle_under_asan_and_ubsan(tmp_path):
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src in ("sched.cpp", "sao.cpp", "ransac.cpp"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run(["g++", "-std=c++17", "-c", os.path.join(CSRC, src), "-o", obj] + SAN + inc,
                       check=True, capture_output=True)
        objs.append(obj)
    obj = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-mpopcnt", "-c", os.path.join(ROOT, "oracle", "chm_oracle.c"),
                    "-o", obj] + SAN, check=True, capture_output=True)
    objs.append(obj)
    exe = str(tmp_path / "host_checks")
    subprocess.run(["g++", "-std=c++17", os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), "-o", exe,
                    "-fopenmp", "-pthread"] + SAN + inc + objs, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "host checks: 0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
