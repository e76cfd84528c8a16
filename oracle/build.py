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
    """Portable build used by the tests (no host-specific instructions, so
    the object runs on any x86-64 host it is copied to)."""
    cmd = ["gcc", "-O3", "-fPIC", "-shared", "-std=c99", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def build_native(outdir, verbose=False) -> str:
    """Build for the host it runs on (-O3 -march=native, OpenMP) into outdir:
    the benchmark's CPU baseline compiles this copy on the machine it times."""
    out = os.path.join(outdir, "_oracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


def build_sanitized(outdir, verbose=False) -> str:
    """AddressSanitizer + UndefinedBehaviorSanitizer build into outdir (the
    tests load it in a child process with the sanitizer runtimes preloaded)."""
    out = os.path.join(outdir, "_oracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
