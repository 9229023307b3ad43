"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the planner
(paper_2509_17257_amd/csrc/planner.cpp) and the oracle (oracle/h2_oracle.c) built with
-fsanitize=address,undefined by g++/gcc (host code only, no GPU code involved) and run on
small random problems (tests/sanitize_main.cpp).  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_planner_and_oracle_under_sanitizers(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g", "-O1"]
    obj = tmp_path / "oracle.o"
    subprocess.run(["gcc", "-std=c99", "-fopenmp", "-ffp-contract=off", *san, "-c",
                    os.path.join(ROOT, "oracle", "h2_oracle.c"), "-o", str(obj)], check=True)
    exe = tmp_path / "sanitized"
    subprocess.run(["g++", "-std=c++17", "-fopenmp", "-ffp-contract=off", *san,
                    os.path.join(ROOT, "tests", "sanitize_main.cpp"),
                    os.path.join(ROOT, "paper_2509_17257_amd", "csrc", "planner.cpp"), str(obj), "-o", str(exe),
                    "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-3000:]
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout
