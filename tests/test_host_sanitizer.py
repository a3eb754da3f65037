"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): the argument checks and status codes of every entry point on a
context without a device, the FP64 finisher (cva_solve_moments, the
symmetric eigensolver) and the Python binding's checks, run by the same
tests as the regular build but on a build whose host objects (api.cpp,
finisher.cpp, pipeline.cpp) are instrumented.  Any sanitizer report aborts
the run, so the bar is a clean pass.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    out = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers(tmp_path):
    asan = _runtime()
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for g++")
    sys.path.insert(0, ROOT)
    from paper_1612_06457_amd.build import build_host_sanitized
    lib = build_host_sanitized(str(tmp_path))
    env = dict(os.environ)
    env.update({"CVAMX_LIB_PATH": lib, "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    probe = ("import ctypes, paper_1612_06457_amd._lib as L; L.lib(); "
             "print(hasattr(ctypes.CDLL(None), '__asan_init'), L.LIB_PATH in open('/proc/self/maps').read())")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.split()[-2:] == ["True", "True"], r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_host_lib.py", "tests/test_binding_checks.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    log = r.stdout + r.stderr
    assert r.returncode == 0, log[-4000:]
    assert "AddressSanitizer" not in log and "runtime error" not in log, log[-4000:]
    assert " passed" in log
