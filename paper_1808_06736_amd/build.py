"""Build libesnufft.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1808_06736_amd.build        # compile every source, link

Every source is compiled on each call; objects go to ``_build/`` next to the
package and the shared library to ``paper_1808_06736_amd/libesnufft.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libesnufft.so")
ARCH = os.environ.get("ESN_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-munsafe-fp-atomics",
          # no packed FP32 instructions in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]

SOURCES = ["params.cpp", "fft.cpp", "plan.cpp", "type3.cpp", "serve.cpp",
           "kernels_sort.hip", "kernels_deconv.hip", "kernels_spread.hip",
           "kernels_interp.hip", "kernels_mfma.hip", "kernels_type3.hip",
           "toeplitz.cpp", "kernels_toeplitz.hip", "kernels_fft.hip", "noalloc.cpp",
           "kernels_mfma2d.hip"]


# Per-source extra flags (none).  The matrix-core kernels keep their MFMA
# accumulators in the accumulation registers, the compiler's default: its
# option to place them in ordinary VGPRs gave MFMA instructions whose result
# registers partly overlap their accumulator input, whose values then depend
# on timing.
EXTRA = {}


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + EXTRA.get(src, []) + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib"]
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
