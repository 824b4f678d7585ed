"""AddressSanitizer and UndefinedBehaviorSanitizer over the host code: the library's planner, validation and ABI
(built with sanitized host code and unchanged GPU code objects) and the C oracle, both run by the CPU tests that
exercise them (planning, plan gate order replayed on the oracle, ABI error paths, oracle pins, measurement oracle).

The sanitized builds live in _build/sanitize and are selected with QS_LIBQS / QS_LIBQS_ORACLE; one LLVM sanitizer
runtime is preloaded into the test process. Any report aborts the run (halt_on_error), so the subprocess must pass.
Leak checking is off: the Python interpreter itself keeps allocations alive at exit.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_host_code_is_clean_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("LLVM sanitizer runtime or hipcc not available")
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    from paper_2203_16044_amd import build as pb
    lib = pb.build_sanitized()
    olib = ob.build_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "QS_LIBQS": lib,
        "QS_LIBQS_ORACLE": olib,
        "PYTHONPATH": ROOT,
    })
    tests = ["tests/test_plan_host.py", "tests/test_abi.py", "tests/test_oracle_pins.py",
             "tests/test_measure_oracle.py", "tests/test_error_metrics.py"]
    # the C consumer links libqs itself (it would need the sanitizer runtime on its link line)
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
           "-k", "not links_from_c", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "passed" in r.stdout
