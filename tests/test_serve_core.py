"""Host-only checks of the request server's arena allocator, launch-region
layout and first-come-first-served admission planner, including an
event-driven simulation with a fake clock (no device)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_16341_amd", "csrc")


def test_serve_core(tmp_path):
    exe = str(tmp_path / "serve_core_check")
    src = os.path.join(ROOT, "tests", "serve_core_check.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-Wall", "-fsanitize=address,undefined",
                    "-I", CSRC, src, "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0 and res.stdout.strip().endswith("OK"), res.stdout + res.stderr
