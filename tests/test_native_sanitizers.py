"""Host C++ of the library built with the address and undefined-behaviour
sanitizers and run on the CPU: the hop-list packer (merging, Hermiticity and
range checks, pair layout, and the Bloch sum it implies against a direct sum
over the raw entries, on hostile and random lists)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_hk_packer_under_sanitizers(tmp_path):
    exe = tmp_path / "hk_pack_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Werror",
           "-I", os.path.join(ROOT, "paper_2312_13051_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "hk_pack_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "checks passed" in out.stdout and "runtime error" not in out.stderr
