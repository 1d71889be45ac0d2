"""Build libbks.so for gfx950 from csrc/ with hipcc (in-tree)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbks.so")
ARCH = os.environ.get("BKS_OFFLOAD_ARCH", "gfx950")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wno-unused-result",
          "-I" + os.path.join(os.path.dirname(HERE), "include")]
# packed FP32 instructions are kept out of the generated code
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def compile_one(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE
    else:
        # host code (plain C++: `-x` applies to the inputs after it), with
        # AVX2 + FMA (every x86-64 host of an MI355X has them)
        cmd = [HIPCC, "-x", "c++", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + [
            "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"), "-mavx2", "-mfma"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-lpthread",
                                                 "-L" + os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas",
                                                 "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
