"""Build step for the HIP library (gfx950), the FP64 instruction-rate
measurement program and, separately, the CPU oracle."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbinv.so")
RATE_EXE = os.path.join(HERE, "mfma_rate")
SOURCES = ["kernels.hip", "batched.hip", "mixed.hip", "levels.hip", "binv_api.hip", "batched_api.hip", "server.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 ops (see the kernels' notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source into libbinv.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose and r.stderr.strip():
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


def build_rate_program() -> str:
    """Compile the standalone FP64 instruction-rate program (always recompiles)."""
    tmp = RATE_EXE + ".tmp"
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [HIPCC, *flags, "-o", tmp, os.path.join(CSRC, "mfma_rate.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, RATE_EXE)
    return RATE_EXE


if __name__ == "__main__":
    print(build_library(verbose=True))
    print(build_rate_program())
