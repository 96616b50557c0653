"""The tuned-shape cache's line format on the CPU (tests/native/tuneline_check.cpp
compiles the library's header with g++ and UBSan and runs its checks)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "tuneline_check.cpp")


def test_tune_cache_line_format(tmp_path):
    exe = str(tmp_path / "tuneline_check")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Werror", "-fsanitize=undefined",
                    "-fno-sanitize-recover=all", "-o", exe, SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("0 failures")
