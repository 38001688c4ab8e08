"""The register-tile kernels' index maps checked on the CPU: builds
tests/index_maps_check.hip as a host program against the kernel headers and
libdqaoa's pass planner, and runs it.  It checks that every layout, in-register
exchange and LDS transpose of the 14-, 13- and 12-qubit tiles is a bijection
that stays inside its buffer and delivers each amplitude where the next
layout expects it, and that the global offsets of every register-tile pass
planned for n <= 34 stay inside the state and cover it once."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2506_10531_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    from paper_2506_10531_amd import _lib
    if not os.path.exists(_lib.SO):
        from paper_2506_10531_amd import build
        build.build()
    exe = str(tmp_path_factory.mktemp("imc") / "index_maps_check")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "index_maps_check.hip"), "-o", exe,
                        "-L" + PKG, "-ldqaoa", "-Wl,-rpath," + PKG],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_index_maps(checker):
    r = subprocess.run([checker], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert r.stdout.startswith("ok "), r.stdout
