"""CPU unit test of the serving loop's host bookkeeping: the first-fit pool
that admits requests against the device-memory budget (filled exactly,
fragmented, coalesced) and the rule that forms a step from pending requests
within a fixed table region (so a step can always be formed when a stream
is free, whatever the requests hold of the budget)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_and_step_rules(tmp_path):
    exe = str(tmp_path / "test_pool")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2406_13881_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "test_pool.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True)
    assert "ok" in out.stdout
