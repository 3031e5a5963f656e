"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The product planner (``csrc/planner.cpp``) and the oracle's C loops (``oracle/srj_oracle.c``)
are each built into a small check program of their own with
``-fsanitize=address,undefined -fno-sanitize-recover=all`` and run; a sanitizer report, or an
invariant the program checks, fails the test.  The two are never linked together.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc/g++")


def _run(cmd, exe, tmp_path):
    subprocess.run(cmd, check=True, cwd=tmp_path)
    # a library preloaded into every process of the machine may precede the ASan runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")


def test_planner_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1511_04292_amd", "csrc")
    exe = str(tmp_path / "planner_check")
    _run(["g++", "-std=c++17", *SAN, f"-I{csrc}", os.path.join(ROOT, "tests", "native", "planner_check.cpp"),
          os.path.join(csrc, "planner.cpp"), "-o", exe], exe, tmp_path)


def test_oracle_loops_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c11", "-ffp-contract=off", *SAN, os.path.join(ROOT, "tests", "native", "oracle_check.c"),
          os.path.join(ROOT, "oracle", "srj_oracle.c"), "-lm", "-o", exe], exe, tmp_path)
