"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The host sources (mesh set-up, layouts, class stencils, P2 stencils, batch
set-up and the C ABI's argument checks) are rebuilt instrumented and linked
with the regular device objects; the host-library tests then run in a child
process with clang's ASan runtime preloaded, so that any out-of-bounds
access, use after free or undefined operation in that code ends the run.
No GPU is needed.
"""
import os
import subprocess
import sys

import pytest

from tests.conftest import ROOT

LIB = os.path.join(ROOT, "paper_2308_01792_amd", "libhytet.so")


@pytest.fixture(scope="module")
def sanitized():
    from paper_2308_01792_amd import _build
    if not os.path.exists(LIB):
        _build.build()
    return _build.build_sanitized(), _build.asan_runtime()


def _env(lib, runtime):
    env = dict(os.environ)
    env.update(HYTET_LIB=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return env


def test_sanitized_library_is_instrumented(sanitized):
    lib, runtime = sanitized
    out = subprocess.run(["nm", "-D", "--undefined-only", lib],
                         capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load8" in out
    assert "__ubsan_handle" in out
    # the child process really loads this build, under the ASan runtime
    code = ("import paper_2308_01792_amd as ht; ht.load(); "
            "maps = open('/proc/self/maps').read(); "
            "assert 'libhytet_san.so' in maps, 'sanitized library not loaded'; "
            "assert 'libclang_rt.asan' in maps, 'ASan runtime not loaded'; "
            "print('ok')")
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT,
                         env=_env(lib, runtime), capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0 and "ok" in res.stdout, res.stderr[-3000:]


def test_host_library_tests_pass_under_sanitizers(sanitized):
    lib, runtime = sanitized
    res = subprocess.run(
        [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
         os.path.join("tests", "test_host_library.py")],
        cwd=ROOT, env=_env(lib, runtime), capture_output=True, text=True,
        timeout=900)
    log = res.stdout[-3000:] + res.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in log, log
    assert "runtime error:" not in log, log
    assert res.returncode == 0, log
