"""The host side of the C-ABI library under AddressSanitizer and UBSan (no GPU).

The host sources (descriptor validation, plan-time tables, workspace arithmetic, error
unwinding of the create/plan calls, including the injected allocation failures) are
rebuilt with -fsanitize=address,undefined on the host compilation only, linked with the
regular kernel objects, and the host boundary tests run against that library in a child
process with clang's sanitizer runtime preloaded.  Any heap overflow, use after free or
undefined behaviour aborts the child.
"""
import os
import subprocess
import sys

import pytest

from paper_2608_28183_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized_library():
    built = os.path.isdir(build.BUILD) and any(f.endswith(".hip.o") for f in os.listdir(build.BUILD))
    if not built:
        pytest.skip("regular build missing: run python -m paper_2608_28183_amd.build first")
    try:
        runtime = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    return build.build_sanitized(), runtime


def test_sanitized_library_is_instrumented(sanitized_library):
    lib, _ = sanitized_library
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load" in syms or "__asan_report_store" in syms
    assert "__ubsan_handle" in syms


def test_host_boundary_tests_under_asan_ubsan(sanitized_library):
    lib, runtime = sanitized_library
    env = dict(os.environ)
    env.update(NLOS_LIBRARY=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
