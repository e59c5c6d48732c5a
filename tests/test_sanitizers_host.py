"""The library's host code under sanitizers, on the CPU: the C-ABI
validation, the 1D operators and bases and the serving scheduler (the .cpp
sources) are compiled with AddressSanitizer + UndefinedBehaviorSanitizer, and
separately with ThreadSanitizer, linked with the unmodified device objects of
the regular build, and driven by tests/c_client/sfhad_host_sanitized.c: every
host path that needs no GPU, including a simulated server fed from two
threads.  Device code is not instrumented (no sanitizer runs on the GPU)."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_11665_amd", "csrc")
OBJ = os.path.join(ROOT, "_build", "sfhad")
ROCM = "/opt/rocm"
HOST_SOURCES = ["capi.cpp", "operators.cpp", "server.cpp"]
DEVICE_OBJECTS = ["dense_kernels", "diag_kernels", "entropy_kernels", "surface_kernels", "curv_kernels",
                  "tensor_kernels", "serve_kernels", "volume_kernels", "volume_kernels_fp32"]
DRIVER = os.path.join(ROOT, "tests", "c_client", "sfhad_host_sanitized.c")


def _build_and_run(tmp, cc, cxx, flags, env):
    objs = [os.path.join(OBJ, o + ".hip.o") for o in DEVICE_OBJECTS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("device objects of the regular build are missing (run the build first)")
    common = ["-O1", "-g", "-fno-omit-frame-pointer", *flags]
    jobs = [[cxx, "-std=c++17", *common, "-D__HIP_PLATFORM_AMD__", "-isystem", os.path.join(ROCM, "include"),
             "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, s), "-o", os.path.join(tmp, s + ".o")]
            for s in HOST_SOURCES]
    jobs.append([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", *common, "-I", os.path.join(ROOT, "include"),
                 "-c", DRIVER, "-o", os.path.join(tmp, "driver.o")])
    with ThreadPoolExecutor(4) as ex:
        for r in ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), jobs):
            assert r.returncode == 0, r.stderr[-3000:]
    exe = os.path.join(tmp, "driver")
    link = [cxx, *flags, "-o", exe, os.path.join(tmp, "driver.o"),
            *[os.path.join(tmp, s + ".o") for s in HOST_SOURCES], *objs,
            "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, cwd=tmp, env={**os.environ, **env})
    assert r.returncode == 0, r.stderr[-6000:]
    assert r.stdout.strip() == "ok"


def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("no host C/C++ compiler")
    _build_and_run(str(tmp_path), "gcc", "g++", ["-fsanitize=address,undefined"],
                   {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})


def test_host_code_under_thread_sanitizer(tmp_path):
    # clang's runtime: it follows condition-variable waits with a deadline
    # (pthread_cond_clockwait), which the host gcc's does not
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    if not os.path.exists(clang):
        pytest.skip("no clang")
    _build_and_run(str(tmp_path), clang, clang + "++", ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
