"""The serving loop's scheduler on the CPU: the state machine of
paper_2606_15650_amd/csrc/sched.hpp with a scripted executor on a fake clock
(tests/native/sched_fake_test.cpp), built with g++ under the address and
undefined-behaviour sanitizers, and its threaded case under the thread
sanitizer.  No GPU and no HIP are involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_fake_test.cpp")
INC = [os.path.join(ROOT, "paper_2606_15650_amd", "csrc"), os.path.join(ROOT, "include")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build_and_run(tmp_path, sanitize: str, args: list[str]) -> str:
    exe = str(tmp_path / f"sched_{sanitize.replace(',', '_')}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitize}",
           "-fno-sanitize-recover=all", *[f"-I{d}" for d in INC], SRC, "-o", exe, "-lpthread"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL PASSED" in r.stdout
    return r.stdout


def test_scheduler_with_fake_executor_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "address,undefined", [])
    for name in ("fifo_results_and_arena", "budget_limits_concurrency", "validation_rejects_malformed_requests",
                 "tickets_and_errors", "stop_with_work_in_flight", "threaded_submitters"):
        assert f"PASS {name}" in out


def test_scheduler_threads_under_tsan(tmp_path):
    _build_and_run(tmp_path, "thread", ["threaded"])
