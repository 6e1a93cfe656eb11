"""Build the C part of the oracle (test infrastructure only).

Compiles ``riccati_ref.c`` into ``oracle/_build/liboracle.so`` with gcc.  The
flags are portable x86-64 (no ``-march=native``) because the built library is
also used on other hosts than the one that built it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "liboracle.so")
SOURCES = [os.path.join(HERE, "riccati_ref.c")]


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def ensure_built():
    if not os.path.exists(LIB_PATH):
        build()
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
