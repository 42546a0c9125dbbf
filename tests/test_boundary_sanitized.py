"""The host-side ABI tests (argument checks, status codes, null handles,
workspace sizes, the host analysis helpers) rerun against a build of
librlb whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer, in a child process with the sanitizer runtime
preloaded: any invalid access, leak-free misuse aside, or undefined
behaviour in the host code aborts the run.  No GPU needed."""
import os
import subprocess
import sys

import pytest

import asan_build

ROOT = asan_build.ROOT


def test_boundary_tests_under_host_sanitizers(tmp_path):
    try:
        rt = asan_build.runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    so = asan_build.build(str(tmp_path))
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, RLB_LIB_PATH=so, LD_PRELOAD=rt + (":" + pre if pre else ""),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child maps the sanitizer runtime and the instrumented library
    probe = ("import ctypes, sys; sys.path.insert(0, %r); from paper_2205_04658_amd import rlb; "
             "L = rlb.lib(); maps = open('/proc/self/maps').read(); "
             "print('asan' in maps and rlb.LIB_PATH in maps and "
             "hasattr(ctypes.CDLL(None), '__asan_init'))" % ROOT)
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("True"), r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", "tests/test_boundary.py", "tests/test_host_analysis.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
