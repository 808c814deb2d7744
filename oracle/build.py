"""Build step for the oracle's shared library (test infrastructure only).

Compiles ``mpref.c`` with the host C compiler into ``libmpref.so`` next to
this file.  Called by the repository's build entry point.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmpref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "mpref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
