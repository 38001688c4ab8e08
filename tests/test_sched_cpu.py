"""The solve queue's scheduling policy on the CPU: tests/sched_check.cpp
drives paper_2506_10531_amd/csrc/sched.h (the admission, step, early-end,
cancellation and bookkeeping decisions that the device queue runs) with a
host backend on a virtual clock, built with AddressSanitizer and
UndefinedBehaviorSanitizer.  It checks FIFO admission within the slots and
the byte budget, back-pressure, cancellation, failed steps, the latency of
an arrival, exact evaluation counts, and that every request's result is
bitwise what it gets alone in the queue."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("g++ is not installed")
    exe = str(tmp_path_factory.mktemp("sched") / "sched_check")
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "sched_check.cpp"),
                        "-o", exe, "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_scheduler_policy_on_a_virtual_clock(checker):
    r = subprocess.run([checker], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert r.stdout.startswith("ok "), r.stdout
