"""Build the HIP library ``librs.so`` (C ABI of ``include/rs.h``) for gfx950.

Every HIP source is compiled with hipcc for ``--offload-arch=gfx950`` only,
with packed FP32 instructions disabled.  The library is written in-tree to
``paper_1510_03110_amd/_build/librs.so``.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD_DIR = os.path.join(PKG, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "librs.so")
SOURCES = ["rs_kernels.hip", "rs_kernels_mfma.hip", "rs_solve.hip", "rs_refine.hip", "rs_large.hip", "rs_mhe.hip",
           "rs_ip.hip", "rs_pad.hip", "rs_static.hip", "rs_capi.cpp"]
HEADERS = ["rs_types.hpp", "rs_device.hpp", "rs_mfma.hpp", "rs_launch.hpp", "rs_vec.hpp"]

# roctx (the ranges the C ABI marks around its calls and kernel launches)
LINK_LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _compile(src, obj, verbose):
    cmd = [hipcc()] + HIPCC_FLAGS + ["-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                     os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l)      # host-pass notice, harmless
    return res.returncode, out


def build(verbose=False):
    """Compile every source to an object (in parallel) and link librs.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = [os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(SOURCES, objs)))
    for (rc, out), src in zip(results, SOURCES):
        if rc != 0:
            sys.stderr.write(out + "\n")
            raise RuntimeError("hipcc failed on %s (%d)" % (src, rc))
        if verbose and out.strip():
            print(out)
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + LINK_LIBS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


# Host sanitizers for the C ABI's own code (plan construction, work tables,
# argument checks), each flag routed to the host compilation only.
SAN_DIR = os.path.join(PKG, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "librs_san.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized(verbose=False):
    """A copy of the library whose host C ABI (rs_capi.cpp) is built with
    AddressSanitizer and UndefinedBehaviorSanitizer, linked with the regular
    objects of every other source (built first if missing).  For host-only
    tests on the CPU, in a process that preloads clang's ASan runtime."""
    objs = [os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES if s != "rs_capi.cpp"]
    if not all(os.path.exists(o) for o in objs):
        build(verbose)
    os.makedirs(SAN_DIR, exist_ok=True)
    obj = os.path.join(SAN_DIR, "rs_capi.o")
    cmd = [hipcc()] + HIPCC_FLAGS + HOST_SAN + ["-g", "-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                                os.path.join(CSRC, "rs_capi.cpp"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + "\n")
        raise RuntimeError("hipcc failed on rs_capi.cpp (sanitized, %d)" % res.returncode)
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + HOST_SAN + \
        ["-Xarch_host", "-shared-libsan"] + objs + [obj] + LINK_LIBS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
