"""Builds libspiir.so (HIP kernels + host library) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libspiir.so")
SOURCES = [os.path.join(CSRC, "spiir_kernels.hip"), os.path.join(CSRC, "spiir_host.cpp")]
ARCH = os.environ.get("SPIIR_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 (v_pk_*_f32) is kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def build_library(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


C_ABI_SRC = os.path.join(ROOT, "tests", "c", "spiir_c_abi.c")
C_ABI_BIN = os.path.join(ROOT, "tests", "c", "spiir_c_abi")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_c_abi(verbose: bool = False) -> str:
    """The torch-free C consumer of the ABI (tests/c), linked against this
    build of libspiir.so and ROCm's HIP runtime."""
    tmp = C_ABI_BIN + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
           "-I", os.path.join(ROCM, "include"), C_ABI_SRC, "-L", PKG, "-lspiir",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1702_02256_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, C_ABI_BIN)
    return C_ABI_BIN


if __name__ == "__main__":
    print(build_library(verbose=True))
