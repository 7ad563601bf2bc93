"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host_asan/drive.cpp calls every entry point of include/cloth.h (plain, batched and
triangle-triangle handles, launch configurations, autotuning, rollouts, surface updates, error
paths) against a stand-in HIP runtime (tests/host_asan/hip_stub.cpp) that performs queued copies
only when the program synchronises, as the runtime may for pageable host memory.  A host buffer
released while a copy of it is still queued is then reported as a use after free.  This is the
regression test for such a release in the batch constructor (the per-slot cloth table), which
crashed a runtime worker thread on the GPU.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_11794_amd", "csrc")
HOST_SOURCES = [os.path.join(CSRC, f + ".cpp")
                for f in ("sim", "host_build", "tiles", "autotune", "rollout")]
TEST_SOURCES = [os.path.join(ROOT, "tests", "host_asan", f) for f in ("drive.cpp", "hip_stub.cpp")]
FLAGS = ["-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_host_paths_clean_under_sanitizers(tmp_path):
    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run(["g++", *FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, HOST_SOURCES + TEST_SOURCES))
    exe = str(tmp_path / "drive")
    r = subprocess.run(["g++", "-fsanitize=address,undefined", *objs, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host paths ok" in r.stdout, r.stdout + r.stderr[-6000:]
