"""Build liboracle.so, the CPU reference (test infrastructure only).

Plain scalar C: -O2, no vector intrinsics, no OpenMP; threads only split the
rows into ranges.  These flags are also what the CPU baseline reports.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CFLAGS = ["-O2", "-fPIC", "-shared", "-pthread", "-fno-tree-vectorize"]


def build(src: str | None = None, out: str | None = None, verbose: bool = False) -> str:
    src = src or os.path.join(HERE, "oracle.c")
    out = out or os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
