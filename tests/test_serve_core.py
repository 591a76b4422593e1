"""Host logic of the serving runtime: admission core built with g++ and run
(no GPU), including under the address and undefined-behaviour sanitizers."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "serve_core_test.cpp")
INC = os.path.join(ROOT, "paper_1810_11966_amd", "csrc")


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined"]])
def test_serve_core(tmp_path, flags):
    exe = tmp_path / "serve_core_test"
    subprocess.run(["g++", "-std=c++17", *flags, "-I", INC, SRC, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all checks passed" in out.stdout
