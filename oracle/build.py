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


SAN_PATH = os.path.join(BUILD_DIR, "liboracle_san.so")


def build(verbose=False, path=None, native=False, sanitize=False):
    """Compile the oracle.  ``native=True`` adds -march=native (for timing the
    oracle on the host that runs it; such a library is not portable),
    ``sanitize=True`` builds it with AddressSanitizer and
    UndefinedBehaviorSanitizer (default path SAN_PATH; load it in a process
    that preloads gcc's ASan runtime), and ``path`` places it elsewhere."""
    out = path or (SAN_PATH if sanitize else LIB_PATH)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    opt = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"] if sanitize else ["-O3"]
    cmd = ["gcc"] + opt + (["-march=native"] if native else []) + ["-std=c99", "-fPIC", "-shared", "-o", tmp] + \
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
