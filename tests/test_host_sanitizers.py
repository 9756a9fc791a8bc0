"""The host runtime and C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with both sanitizers on its host pass (device code as
usual, build.py --sanitize) and the host-side ABI tests are run against that
build in a child process with the sanitizer runtime preloaded: argument
validation, the star-description checks, struct layouts and exports.  Any
out-of-bounds access, use after free or undefined behaviour in those paths
ends the child with a sanitizer report and fails this test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2301_04259_amd")
CSRC = os.path.join(PKG, "csrc")

pytestmark = pytest.mark.skipif(
    shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not available"
)


def _build_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("soap_build", os.path.join(PKG, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(ROOT, "include", "soap.h")]
    return any(os.path.getmtime(s) > t for s in srcs)


@pytest.fixture(scope="module")
def san_lib():
    b = _build_module()
    lib = b.SAN_LIB
    if _stale(lib):
        b.build_sanitized()
    return lib, b.san_runtime()


def test_sanitized_build_is_instrumented(san_lib):
    lib, _ = san_lib
    und = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in und or "__asan_report_load4" in und
    assert "__ubsan_handle_" in und


def test_host_abi_checks_clean_under_asan_and_ubsan(san_lib):
    lib, rt = san_lib
    env = dict(os.environ)
    env.update(
        LD_PRELOAD=rt,
        SOAP_LIB=lib,
        ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
        UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
    )
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
         os.path.join(ROOT, "tests", "test_abi_host.py")],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=600,
    )
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
