"""Host constants that every MSD decision depends on (csrc/trig_bounds.hpp),
built with g++ and run on the CPU: the threshold folding checked exhaustively
near its cut, the basis-form pair bound likewise, and the written-out fit's
pruning bounds on triplets built to pass or to sit on the cut (paper Sec. 3.2,
step 2)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "bounds_test.cpp")
INC = os.path.join(ROOT, "paper_1810_11966_amd", "csrc")


def test_folding_pair_and_fit_bounds(tmp_path):
    exe = tmp_path / "bounds_test"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I", INC, SRC, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all checks passed" in out.stdout
