"""Build the C oracle (oracle.c) into oracle/_oracle.so with gcc.

Test infrastructure only: the shared object is loaded by the tests, the smoke
check and the benchmark's CPU-baseline leg, never by the product library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
OUT = os.path.join(HERE, "_oracle.so")


def build(verbose=False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
