"""The host logic of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.

libakra_san.so is the library with its host code instrumented (device code unchanged), built beside
libakra.so.  The host-only tests (null plans, argument and size validation, option defaults, exported
symbols) run in a child process against it with the clang ASan runtime preloaded; any sanitizer
report ends the child with a failure.  No GPU is needed: these paths return before the device is
touched."""
import os
import subprocess
import sys

import pytest

from paper_2606_06175_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _need_san():
    if not os.path.exists(B.LIB_SAN):
        pytest.skip("libakra_san.so is not built (run __graft_entry__.build())")
    rt = B.asan_runtime()
    if rt is None:
        pytest.skip("the clang AddressSanitizer runtime is not installed")
    return rt


def test_sanitized_build_is_instrumented():
    _need_san()
    out = subprocess.run(["nm", "-D", "--undefined-only", B.LIB_SAN], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in out or "__asan_report_load_n" in out
    assert "__ubsan_handle_" in out
    plain = subprocess.run(["nm", "-D", "--undefined-only", B.LIB], capture_output=True, text=True).stdout
    assert "__asan_" not in plain


def test_host_logic_under_sanitizers():
    rt = _need_san()
    env = dict(os.environ, LD_PRELOAD=rt, AKRA_LIBRARY=B.LIB_SAN,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    probe = ("from paper_2606_06175_amd import akra; import ctypes; "
             "assert akra.LIB_PATH.endswith('libakra_san.so'); "
             "assert hasattr(ctypes.CDLL(None), '__asan_init'); print('sanitized library in use')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "sanitized library in use" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_capi_host.py",
                        "tests/test_capi_symbols.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-500:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-3000:]
