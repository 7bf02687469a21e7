"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The three HIP sources are compiled with the sanitizers on the host side only
(device code as usual, at -O1 to keep the build short), linked with the
checks of ``host_sanitize/host_checks.cpp`` (geometry validation and
workspace sizes over a seeded sweep, argument and parameter checks, error
paths with no device present), and run; any sanitizer report ends the run
with a non-zero status.  CPU only: the checks need no GPU."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_01444_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_host_code_under_asan_and_ubsan(tmp_path):
    objs = []

    def compile_one(name):
        obj = str(tmp_path / f"{name}.o")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", *HOST_SAN, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, f"{name}.hip"),
               "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(3) as ex:
        objs = list(ex.map(compile_one, ["lbm_api", "lbm_batch_api", "lbm3d_api"]))
    drv = str(tmp_path / "host_checks")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", *san, "-I", INCLUDE,
                        os.path.join(HERE, "host_sanitize", "host_checks.cpp"), *objs, "-o", drv,
                        "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "host checks: ok" in r.stdout, r.stderr[-4000:]
