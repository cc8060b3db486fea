"""Build the gfx950 shared library liblbm.so in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # fused multiply-adds only within one source expression (decided by the front end, so
    # every instantiation of a stage body, single case or batched, rounds identically); code
    # that needs a product rounded on its own says so with `#pragma clang fp contract(off)`
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "csrc", f) for f in ("lbm_api.hip", "nn_api.hip")]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPFLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
