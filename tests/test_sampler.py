"""The kernel-family timer's launch sampler under concurrent host threads
(the pairs of a batched registration launch from several threads): built
from its host-only header with g++ and ThreadSanitizer, no GPU.  Each
launch's sampling decision must reach the events of that same launch."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_sampler_decisions_stay_with_their_thread(tmp_path):
    exe = str(tmp_path / "sampler_threads")
    src = os.path.join(ROOT, "tests", "sampler_threads.cpp")
    inc = os.path.join(ROOT, "paper_1807_11560_amd", "csrc")
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=thread", "-I", inc, src,
                            "-o", exe], capture_output=True, text=True)
    if build.returncode != 0 and "sanitizer" in build.stderr.lower():
        pytest.skip("ThreadSanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(run.stdout)
    assert "ThreadSanitizer" not in run.stderr, run.stderr[-2000:]
    assert run.returncode == 0, run.stdout + run.stderr[-2000:]
