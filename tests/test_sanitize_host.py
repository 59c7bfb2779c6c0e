"""The library's host code (plan building: validation, relabelling, column
slices, work maps, the Lanczos estimate) under AddressSanitizer and
UndefinedBehaviorSanitizer.  CPU only: the library is rebuilt with the
sanitizers on its host code only, and tests/sanitize_plan_driver.cpp drives
cpaa_plan on graphs of several shapes with every option that changes that code.
Without a GPU each valid plan stops at its first device allocation."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

# sanitizers on the host side of every translation unit (never on device code)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
# a low cap on the packed entries of the column-sliced layout (int32 offsets in
# the product build), so that the driver reaches the guard with small graphs
ENTRY_LIMIT = ["-DCPAA_TEST_SLICE_ENTRY_LIMIT=100000"]


@pytest.mark.slow
def test_plan_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2112_01743_amd import build as B
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(B.HIPCC) or not os.path.exists(clang):
        pytest.skip("ROCm toolchain not found")
    objs = []
    procs = []
    for src in B.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [B.HIPCC, *B.FLAGS, "-O1", *HOST_SAN, *ENTRY_LIMIT, "-c", os.path.join(B.CSRC, src),
               "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                            text=True)))
        objs.append(obj)
    for src, pr in procs:
        out, _ = pr.communicate()
        assert pr.returncode == 0, f"{src}:\n{out}"
    lib = str(tmp_path / "libcpaa_san.so")
    subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, "-o", lib,
                    *objs], check=True, capture_output=True)
    exe = str(tmp_path / "plan_driver")
    subprocess.run([clang, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", *ENTRY_LIMIT,
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize_plan_driver.cpp"), lib,
                    "-Wl,-rpath," + str(tmp_path), "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(res.stdout[-4000:], res.stderr[-4000:])
    assert res.returncode == 0 and "ALL OK" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
