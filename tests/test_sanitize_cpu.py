"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the translation units that carry host logic (context and
planner, solve queue, COBYLA, outer cycle, sampled objective) are rebuilt
with both sanitizers on their host code and linked with the regular objects
of the kernel units, and tests/sanitize_driver.py drives every host-side
path on a host-only context in a child process.  Any sanitizer report
aborts the child."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_10531_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_UNITS = ("capi", "queue", "cobyla", "cycle", "objective")
KERNEL_UNITS = ("fwd14", "fwd13d", "grad12", "grad13", "kernels", "small")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _kernel_objects():
    """The regular build's objects of the kernel units, rebuilt if stale."""
    from paper_2506_10531_amd import build
    objs = [os.path.join(ROOT, "_build", u + ".hip.o") for u in KERNEL_UNITS]
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    newest = max(os.path.getmtime(f) for f in srcs)
    if not all(os.path.exists(o) and os.path.getmtime(o) >= newest for o in objs):
        build.build()
    return objs


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc is not installed")
    out = tmp_path_factory.mktemp("san")
    base = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]

    def compile_unit(u):
        o = str(out / (u + ".o"))
        r = subprocess.run(base + SAN + ["-c", os.path.join(CSRC, u + ".hip"), "-o", o],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return o

    with ThreadPoolExecutor(max_workers=len(HOST_UNITS)) as ex:
        objs = list(ex.map(compile_unit, HOST_UNITS))
    so = str(out / "libdqaoa_san.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                        "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", so,
                        *objs, *_kernel_objects(), "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return so


def test_host_paths_clean_under_asan_and_ubsan(sanitized_lib):
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    assert os.path.exists(rt), rt
    env = dict(os.environ, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_driver.py"),
                        sanitized_lib], capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout[-2000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert r.stdout.startswith("ok "), report
