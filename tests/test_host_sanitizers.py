"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the host ABI tests (argument checks, parameter
validation, null handling, error text; no device) run again in a child
process against the instrumented build of the same sources, with the ASan
runtime preloaded.  Any sanitizer report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1908_02456_amd import build as B  # noqa: E402


@pytest.fixture(scope="module")
def hostsan_env():
    if not os.path.exists(B.ASAN_RUNTIME):
        pytest.skip("no ASan runtime in this toolchain")
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(ROOT, "include", "abc_dtn.h")]
    newest = max(os.path.getmtime(s) for s in srcs)
    if not os.path.exists(B.HOSTSAN_LIB) or os.path.getmtime(B.HOSTSAN_LIB) < newest:
        B.build_host_sanitized()
    env = dict(os.environ)
    env.update(LD_PRELOAD=B.ASAN_RUNTIME, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", ABC_DTN_LIBRARY=B.HOSTSAN_LIB)
    return env


def test_instrumented_library_is_the_one_loaded(hostsan_env):
    nm = subprocess.run(["nm", "-D", "--undefined-only", B.HOSTSAN_LIB], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in nm and "__ubsan_handle_" in nm
    code = ("from paper_1908_02456_amd import _lib; _lib.load(); "
            "print(open('/proc/self/maps').read())")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=hostsan_env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert B.HOSTSAN_LIB in r.stdout
    assert "libclang_rt.asan" in r.stdout


def test_host_abi_tests_pass_under_sanitizers(hostsan_env):
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_host.py"), "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=hostsan_env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
