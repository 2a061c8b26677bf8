"""The library's host code (graph upload and validation, the batched pass
driver, the server's admission, slots, memory pool and worker threads) built
against a host-only stand-in for the HIP runtime and run under
AddressSanitizer and ThreadSanitizer (no GPU needed)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "cpu_sim")
CSRC = os.path.join(ROOT, "paper_2205_14503_amd", "csrc")


@pytest.mark.parametrize("sanitizer", ["address", "thread"])
def test_host_logic_under_sanitizer(tmp_path, sanitizer):
    exe = str(tmp_path / f"sim_{sanitizer}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-fno-omit-frame-pointer",
           "-I" + SIM, "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), "-x", "c++",
           os.path.join(CSRC, "engine.cpp"), os.path.join(CSRC, "pass.cpp"), os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "noalloc.cpp"),
           os.path.join(SIM, "fake_runtime.cpp"), os.path.join(SIM, "server_driver.cpp"), "-lpthread", "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "cpu_sim ok" in res.stdout
