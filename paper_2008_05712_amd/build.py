"""Build libgcharm.so (hipcc, gfx950) in-tree beside this file."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgcharm.so")

HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
               # packed FP32 instructions stay disabled; the compiler emits plain v_fma_f32 / v_mul_f32
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               # every atomic here is issued by one lane; left to the atomic optimizer, the returned
               # value is broadcast at once, which waits for the atomic where it is issued (the
               # whole-step kernel requests its next ticket early and reads it only at the end)
               "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
               "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
           "-o", tmp, *srcs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
