"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The host-side library tests (block enumeration, contraction planning, SU(2)
bookkeeping and recoupling scalars, error codes, planner properties, the
scatter epilogue's tables) run in a
child process against a second build of libsymten whose host code carries
both sanitizers (device code as usual, never launched here).  Any report
fails the test: UBSan is built not to recover, ASan halts on its first error.
Leak checking is off, since the interpreter itself keeps memory until exit."""
import os
import subprocess
import sys

from paper_1808_10804_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_lib_host.py", "tests/test_lib_su2_host.py", "tests/test_planner_property_host.py",
              "tests/test_scatter_tables_host.py"]


def test_host_tests_pass_under_asan_and_ubsan():
    lib = build.build_sanitized()
    env = dict(os.environ)
    env["SYMTEN_LIB"] = lib
    env["LD_PRELOAD"] = " ".join(p for p in (build.asan_runtime(), env.get("LD_PRELOAD", "")) if p)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *HOST_TESTS],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=1500)
    out = r.stdout
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out, out[-2000:]
