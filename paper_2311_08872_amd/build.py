"""Build the gfx950 library ``libdk_mlmc.so`` in-tree with hipcc.

Every HIP translation unit is compiled for gfx950 only, with packed-FP32 instructions
disabled and with correctly rounded FP32 division and square root wherever the source writes
them (the Gaussian transform's radius root is formed correctly rounded by its own sequence;
the remaining FP32 roots and quotients, e.g. of the FP32 Fourier and semi-implicit kernels,
take the compiler's correctly rounded ones).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdk_mlmc.so")

SOURCES = ["dk_kernels.hip", "dk_round.hip", "dk_stream.hip", "dk_fourier.hip", "dk_theta.hip", "dk_cnn.hip",
           "dk_noalloc.hip", "dk_host_common.cpp", "dk_levels.cpp", "dk_tuning.cpp", "dk_rounds.cpp", "dk_alg1.cpp",
           "dk_samplers.cpp", "dk_arena.cpp", "dk_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fhip-fp32-correctly-rounded-divide-sqrt",
          "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd, cwd=BUILD)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs, cwd=BUILD)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
