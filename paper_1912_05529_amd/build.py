"""Builds libmig.so (all HIP sources, gfx950) in the package directory."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmig.so")

# Packed FP32 VALU instructions are disabled on purpose (-packed-fp32-ops):
# every FP32 operation is a plain VOP instruction.
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build_lib(out: str = LIB, extra: list[str] | None = None, verbose: bool = False) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", *HIPFLAGS, "-I", os.path.join(ROOT, "include"),
           *(extra or []), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_lib(verbose=True))
