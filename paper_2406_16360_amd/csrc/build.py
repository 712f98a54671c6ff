"""Compile the gfx950 HIP library libmirres.so (in-tree, next to the package)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
LIB = os.path.join(PKG, "libmirres.so")
SOURCES = ["bvh.hip", "render.hip", "denoise.hip", "field.hip", "sort.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed-FP32 instructions stay off (they have given silent wrong results on these boxes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",          # hardware float atomics for the gradient scatter
    # fp32 division and square root as reciprocal/multiply and the hardware
    # square root (about 1 ulp) instead of the correctly rounded sequences
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-Wno-unused-result",
]


# measured memory ceilings for the benchmark's roofline report (not part of the renderer)
ROOFS_LIB = os.path.join(PKG, "libmrsroofs.so")
ROOFS_SOURCES = ["roofs.hip"]


def _compile(sources, out, verbose):
    cmd = ["hipcc", *FLAGS, *[os.path.join(HERE, s) for s in sources], "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _compile(SOURCES, LIB, verbose)
    _compile(ROOFS_SOURCES, ROOFS_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
