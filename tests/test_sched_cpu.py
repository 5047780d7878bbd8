"""Admission policy of the request server, checked on the CPU (g++ build of
the policy header; no GPU involved)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy(tmp_path):
    exe = str(tmp_path / "sched_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    "-o", exe, os.path.join(ROOT, "tests", "sched_check.cpp")], check=True)
    p = subprocess.run([exe], capture_output=True, text=True)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "ok" in p.stdout
