"""Build the HIP library (libbl.so) in-tree for gfx950 with hipcc."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libbl.so")
SOURCES = [os.path.join(PKG, "csrc", n) for n in ("eval.hip", "sur.hip", "peaks.hip", "host.cpp")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
         # Packed FP32 instructions stay off: some of their forms gave wrong results, with no error.
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    """Compile every source into libbl.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + ["-I", os.path.join(ROOT, "include")] + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
