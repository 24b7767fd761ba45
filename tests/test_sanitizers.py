"""AddressSanitizer / UndefinedBehaviorSanitizer builds, on the CPU, of the
host-side index arithmetic: the library's graph plans (csrc/plan.hpp, the
in-CSR of both models, the equal-weight form, the count-threshold planes and
the sweep's node batches, each checked against a brute-force recomputation)
and the CPU oracle (every output consistent on random graphs and edge
cases).  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, compiler, sources, extra, name, libs=()):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / name)
    cmd = [compiler, *SAN, *extra, "-o", exe, *sources, *libs]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    return res.stdout


def test_plan_builders_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++", [os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp")],
                         ["-std=c++17", "-I", os.path.join(ROOT, "paper_2404_17059_amd", "csrc")], "plan_check")
    assert "plan_check ok" in out


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
                                           os.path.join(ROOT, "oracle", "imsim_oracle.c")],
                         ["-std=c11", "-Wno-unknown-pragmas"], "oracle_check", libs=["-lm"])
    assert "oracle_check ok" in out
