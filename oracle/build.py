"""Compile the oracle's C source into oracle/liboracle.so with gcc (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src: str = None, out: str = None) -> str:
    """Compile lbm_oracle.c (or another copy of it, `src`) into liboracle.so (or `out`)."""
    src = src or os.path.join(HERE, "lbm_oracle.c")
    out = out or LIB
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-I", HERE, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
