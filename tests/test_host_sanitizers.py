"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host_sanitize_driver.cpp calls every host entry point of the C ABI
(network validation, preparation with every reduction, grouping, weight,
sampling and layout option, plan queries, export, targets, estimators and the
two-state diagnosis) on seeded random networks and on invalid inputs.  It is
compiled with g++ together with the host sources (no device code) and must
finish without a sanitizer report or a failed check.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1605_00854_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_entry_points_are_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    srcs = [os.path.join(CSRC, f) for f in ("host_net.cpp", "host_plan.cpp", "host_stats.cpp")]
    srcs.append(os.path.join(HERE, "host_sanitize_driver.cpp"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC] + srcs + ["-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "0 failures" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
