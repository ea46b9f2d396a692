"""The library's host-only logic (plan validation and workspace layout, serving arena and
admission: paper_2008_01340_amd/csrc/ntt_host.cpp) built as plain C++ with
AddressSanitizer and UndefinedBehaviorSanitizer, and exercised by tests/host_check.cpp
over 20,000 random plan configurations and random arena / admission sequences checked
against a bitmap model.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_host_logic_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_check")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-I" + os.path.join(ROOT, "include"),
             os.path.join(ROOT, "tests", "host_check.cpp"),
             os.path.join(ROOT, "paper_2008_01340_amd", "csrc", "ntt_host.cpp"), "-o", exe]
    res = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe, "20000"], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ok"), run.stdout
    laid, refused = (int(x) for x in run.stdout.split("plans: ")[1].split(" laid out, ")[0:1] +
                     run.stdout.split(" laid out, ")[1].split(" refused")[0:1])
    assert laid > 5000 and refused > 1000
