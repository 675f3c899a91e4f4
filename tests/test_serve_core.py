"""Host tests of the serving scheduler (admission by footprint, resident plan
tables with eviction, continuous batching) against a fake device, built with
g++ under the address/undefined-behaviour and the thread sanitizers."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "serve_core_test.cpp")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_serve_core(tmp_path, san):
    exe = str(tmp_path / "serve_core_test")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={san}", "-fno-omit-frame-pointer", SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
