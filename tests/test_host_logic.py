"""Host logic of libbks without a GPU: the work schedules of the
tensor-times-block kernels (every stored entry processed exactly once, split
segments summed through the fixed-order tree) and the host dense kernels of
the inner solve (register-blocked product, blocked Cholesky, symmetric
eigensolver and its leading-eigenvector path; results independent of the
thread count), and the inner
solve's device interface (a plain-loop implementation of its contract gives
the same solution as the host products).  Compiles
tests/cpp/host_logic.cpp with the library's host sources and runs it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_07595_amd", "csrc")


# host-only builds (g++, no device code): the plain optimised build, and one
# with AddressSanitizer and UBSan that fails on any out-of-bounds access,
# leak or undefined behaviour in the host sources
BUILDS = {
    "plain": ["-O2"],
    "sanitized": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"],
}


@pytest.mark.parametrize("build", sorted(BUILDS))
def test_host_logic(tmp_path, build):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "host_logic")
    cmd = [cxx] + BUILDS[build] + ["-std=c++17", "-mavx2", "-mfma", "-pthread", "-I", CSRC,
           os.path.join(ROOT, "tests", "cpp", "host_logic.cpp"),
           os.path.join(CSRC, "schedule.cpp"), os.path.join(CSRC, "linalg.cpp"),
           os.path.join(CSRC, "scale.cpp"),
           os.path.join(CSRC, "inner.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("schedule", "group_schedule", "scale", "wide_schedule", "fix_tree", "dgemm",
                 "cholesky_threads", "sym_eig", "top_eigvecs", "inner_device"):
        assert f"ok {name}" in r.stdout


def test_upload_formats(tmp_path):
    """The tensor upload's host code (canonicalisation, merging of repeated
    positions, validation, the slice-major and pair layouts and the pair-row
index)
    against an ordered-map construction of the same layouts, with the HIP
    runtime calls it makes replaced by host memory; built with
    AddressSanitizer + UBSan (host code only, g++)."""
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime.h")):
        pytest.skip("no HIP headers")
    exe = str(tmp_path / "format_host")
    cmd = [cxx] + BUILDS["sanitized"] + ["-std=c++17", "-mavx2", "-mfma", "-pthread",
                                         "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
                                         "-I", CSRC,
                                         os.path.join(ROOT, "tests", "cpp", "format_host.cpp"),
                                         os.path.join(CSRC, "format.cpp"),
                                         os.path.join(CSRC, "scale.cpp"),
                                         os.path.join(CSRC, "linalg.cpp"),
                                         os.path.join(CSRC, "schedule.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("random", "distinct", "full_symmetric", "validation", "scaling"):
        assert f"ok formats_{name}" in r.stdout
