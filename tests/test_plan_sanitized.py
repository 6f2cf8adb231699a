"""The host pre-factorisation (plan.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only) and driven over a grid of
plan shapes by tests/sanitize_plan.cpp: any out-of-bounds access, use after
free, overflow or other undefined behaviour in its index arithmetic aborts
the driver with a report."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_plan_factorisation_under_asan_ubsan():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_plan")
        cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", os.path.join(ROOT, "paper_2101_02286_amd", "csrc", "plan.cpp"),
               os.path.join(ROOT, "tests", "sanitize_plan.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
        built = int(out.split("plans built")[1].split()[0])
        assert built > 5000
