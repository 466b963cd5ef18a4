"""Build libfsr.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2202_13926_amd.build

The library holds the C ABI of include/fsr.h; the Python binding in this
package loads it with ctypes.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfsr.so")

SOURCES = ["fsr_api.cpp", "fsr_batched.cpp", "fsr_serve.cpp", "fsr_plain.hip", "fsr_plain_sg.hip",
           "fsr_batched.hip", "fsr_reuse.hip"]
HEADERS = ["fsr_device.h", "fsr_block.h", "fsr_block_sg.h", "fsr_block_s24.h", "fsr_block_multi.h", "fsr_block_split4.h", "fsr_mfma.h", "fsr_internal.h",
           "fsr_batch_internal.h", "fsr_runtime.h", "fsr_sched.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-fvisibility=hidden", "-Wall",
    # packed FP32 instructions stay off: the scalar forms are what is validated
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs: the DFT's accumulators are
    # short-lived, and AGPR copies would push the kernel past 168 registers
    # (three wavefronts per SIMD)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every source into paper_2202_13926_amd/libfsr.so (always rebuilds)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if noise not in ln and "argument unused during compilation: '--hip-link'" not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
