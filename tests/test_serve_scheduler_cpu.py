"""The serving scheduler (csrc/serve_core.h) on the CPU, behind a fake
executor: admission by memory under the arena cap, FIFO order with
head-of-line blocking, the per-launch GEMM cap, failed launches and failed
completions, drain on stop, kept outputs and their release.  The harness
is plain C++ (no HIP), built with g++ here: plainly, with the address and
undefined-behaviour sanitizers, and with the thread sanitizer (the
scheduler thread and the submitting threads share its state)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


SANITIZERS = {"plain": [], "asan_ubsan": ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"],
              "tsan": ["-fsanitize=thread"]}


@pytest.mark.parametrize("san", sorted(SANITIZERS))
def test_scheduler_behind_fake_executor(tmp_path, san):
    exe = str(tmp_path / ("fake_exec_test_" + san))
    src = os.path.join(HERE, "serve_core", "fake_exec_test.cpp")
    inc = os.path.join(ROOT, "paper_2208_09822_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-pthread"] + SANITIZERS[san] +
                          ["-I", inc, src, "-o", exe])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout
    assert r.stdout.count("ok ") >= 18
