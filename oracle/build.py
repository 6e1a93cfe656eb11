"""Build the C part of the oracle (test infrastructure only).

Compiles ``riccati_ref.c`` into ``oracle/_build/liboracle.so`` with gcc.  The
default flags are portable x86-64 (no ``-march=native``) because the built
library is also used on other hosts than the one that built it; the timed
CPU baseline builds a host-tuned copy where it runs.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "liboracle.so")
SOURCES = [os.path.join(HERE, "riccati_ref.c")]


def build(verbose=False, path=None, native=False):
    """Compile the oracle.  ``native=True`` adds -march=native (for timing the
    oracle on the host that runs it; such a library is not portable), and
    ``path`` places it elsewhere than the default library."""
    out = path or LIB_PATH
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3"] + (["-march=native"] if native else []) + ["-std=c99", "-fPIC", "-shared", "-o", tmp] + \
        SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def ensure_built():
    if not os.path.exists(LIB_PATH):
        build()
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
