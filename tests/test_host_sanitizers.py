"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The host side of the C ABI (plan construction, leaf and tree tables,
receding-horizon and split layouts, argument checks) is built with both
sanitizers into a copy of the library, and the plan and ABI tests run
against it in a process that preloads clang's ASan runtime; the C oracle
is built the same way with gcc and its pins run against it.  Any report
(invalid access, overflow, undefined behaviour) ends the process with an
error.  The device code is not instrumented (GPU sanitizers are not used)."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHECK = """
import os, sys
maps = open('/proc/self/maps').read()
assert {runtime!r} in maps, 'sanitizer runtime not loaded'
{load}
assert {lib!r} in open('/proc/self/maps').read(), 'sanitized library not loaded'
import pytest
sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not gpu'] + {tests!r}))
"""


def _run(runtime, env_extra, load, lib, tests):
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", **env_extra)
    code = CHECK.format(runtime=os.path.basename(runtime), load=load, lib=lib, tests=tests)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=900)
    out = r.stdout
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out


def test_host_abi_plans_under_sanitizers():
    runtimes = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not runtimes:
        pytest.skip("clang ASan runtime not installed")
    from paper_1510_03110_amd import build as b
    lib = b.build_host_sanitized()
    load = "from paper_1510_03110_amd import rs; rs.library()"
    _run(runtimes[-1], {"RS_LIBRARY": lib}, load, os.path.basename(lib),
         ["tests/test_plan.py", "tests/test_abi.py"])


def test_oracle_under_sanitizers():
    runtime = subprocess.run(["gcc", "-print-file-name=libasan.so"], stdout=subprocess.PIPE, text=True).stdout.strip()
    if not os.path.isabs(runtime) or not os.path.exists(runtime):
        pytest.skip("gcc ASan runtime not installed")
    from oracle import build as ob
    lib = ob.build(sanitize=True)
    load = "from oracle import riccati; riccati._load()"
    tests = sorted(os.path.relpath(p, ROOT) for p in glob.glob(os.path.join(ROOT, "tests", "test_oracle*.py")))
    _run(runtime, {"ORACLE_LIBRARY": lib}, load, os.path.basename(lib), tests)
