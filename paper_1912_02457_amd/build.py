"""Builds the gfx950 HIP library ``lib/libswe_hip.so`` in-tree with hipcc."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/swe_kernels.hip", "csrc/swe_api.hip", "csrc/swe_ensemble.hip", "csrc/swe_server.hip",
           "csrc/swe_preprocess.hip"]
LIB = os.path.join(HERE, "lib", "libswe_hip.so")
ARCH = os.environ.get("SWE_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b+c only within one expression: every inlined copy of the same
    # source expression rounds the same way, so interior and edge tiles (and
    # hence any tiling) give bitwise identical results
    "-ffp-contract=on",
]


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *[os.path.join(HERE, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
